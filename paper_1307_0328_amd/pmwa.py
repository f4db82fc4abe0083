"""ctypes binding of libpmwa.so (include/pmwa.h): argument marshalling only.

Every step of the sweep runs in the HIP kernels of the library; there is no
fallback.  If the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmwa.so")

PMWA_OK, PMWA_EINVAL, PMWA_ENOMEM, PMWA_EDEVICE, PMWA_EOVERFLOW, PMWA_ESTATE = 0, -1, -2, -3, -4, -5
PH_V, PH_R, PH_S, PH_BT, PH_BSX, PH_BSY, PH_END = 1, 2, 3, 4, 5, 6, 7

EXPORTS = ["pmwa_create", "pmwa_sweep", "pmwa_phase", "pmwa_measure", "pmwa_status",
           "pmwa_get_state", "pmwa_set_state", "pmwa_chain_info", "pmwa_default_event_cap",
           "pmwa_destroy", "pmwa_strerror", "pmwa_set_timing", "pmwa_set_timing_phases", "pmwa_phase_times", "pmwa_diag",
           "pmwa_green", "pmwa_chain_status", "pmwa_observables", "pmwa_reset_observables",
           "pmwa_state_hash", "pmwa_slot_fits", "pmwa_green_static", "pmwa_correlator",
           "pmwa_create_slots", "pmwa_slot_load", "pmwa_slot_release", "pmwa_slot_progress",
           "pmwa_worms_general"]


class pmwa_params(C.Structure):
    _fields_ = [("Lx", C.c_int32), ("Ly", C.c_int32), ("beta", C.c_double),
                ("t", C.c_double), ("V", C.c_double), ("mu", C.c_double), ("eta", C.c_double),
                ("dom_x", C.c_int32), ("dom_y", C.c_int32), ("dom_tau", C.c_int32),
                ("ticks_log2", C.c_int32), ("n_cycle", C.c_int32), ("C", C.c_double),
                ("seed", C.c_uint64), ("chain_id", C.c_uint32), ("pad_", C.c_uint32)]


class pmwa_opts(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("scatter_mode", C.c_int32), ("series_cap", C.c_int32),
                ("event_cap", C.c_int32), ("use_graph", C.c_int32), ("regen_mode", C.c_int32),
                ("vertex_mode", C.c_int32), ("scatter_lds", C.c_int32), ("groups", C.c_int32),
                ("vertex_rows", C.c_int32)]


class pmwa_obs(C.Structure):
    _fields_ = [("nv", C.c_int64), ("nkink", C.c_int64), ("nw", C.c_int64),
                ("occ2", C.c_int64), ("nn2", C.c_int64), ("qimp", C.c_double)]


class pmwa_summary(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("sweeps", "nv", "nkink", "nw", "occ2", "nn2")] + \
               [(n, C.c_double) for n in ("qimp", "nv_sq", "nkink_sq", "nw_sq", "occ2_sq", "nn2_sq",
                                          "qimp_sq", "E", "E_alt", "E_eta", "density", "Q", "Q_imp",
                                          "b", "err_E", "err_density", "err_Q", "err_Q_imp")]


GQ_DMAX, GQ_AMAX, GQ_CAPMAX = 8, 4, 255


class pmwa_localq(C.Structure):
    _fields_ = [("d", C.c_int32), ("nalpha", C.c_int32),
                ("q", C.c_double * (GQ_AMAX * GQ_DMAX * GQ_DMAX))]


class pmwa_info(C.Structure):
    _fields_ = [("C", C.c_double), ("rho_max", C.c_double), ("delta", C.c_double),
                ("lam", C.c_double), ("n_cycle", C.c_int32), ("M", C.c_int32),
                ("event_cap", C.c_int32), ("bond_cap", C.c_int32), ("n_domains", C.c_int64)]


OBS_DTYPE = np.dtype([("nv", "<i8"), ("nkink", "<i8"), ("nw", "<i8"),
                      ("occ2", "<i8"), ("nn2", "<i8"), ("qimp", "<f8")])

_lib = None


def lib():
    """Load libpmwa.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1307_0328_amd/build.py "
                               "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.pmwa_create.argtypes = [P(pmwa_params), C.c_int, P(pmwa_opts), P(C.c_void_p)]
        L.pmwa_sweep.argtypes = [C.c_void_p, C.c_int64]
        L.pmwa_phase.argtypes = [C.c_void_p, C.c_int]
        L.pmwa_measure.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int64, P(C.c_int64)]
        L.pmwa_status.argtypes = [C.c_void_p]
        L.pmwa_get_state.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_int64, P(C.c_int64), P(C.c_uint64)]
        L.pmwa_set_state.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_int64, C.c_uint64]
        L.pmwa_chain_info.argtypes = [C.c_void_p, C.c_int, P(pmwa_info)]
        L.pmwa_default_event_cap.argtypes = [P(pmwa_params)]
        L.pmwa_destroy.argtypes = [C.c_void_p]
        L.pmwa_destroy.restype = None
        L.pmwa_set_timing.argtypes = [C.c_void_p, C.c_int]
        L.pmwa_set_timing_phases.argtypes = [C.c_void_p, C.c_uint32]
        L.pmwa_phase_times.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.pmwa_diag.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int]
        L.pmwa_green.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_void_p]
        L.pmwa_create_slots.argtypes = [P(pmwa_params), C.c_int, P(pmwa_opts), P(C.c_void_p)]
        L.pmwa_slot_load.argtypes = [C.c_void_p, C.c_int, P(pmwa_params), C.c_int64]
        L.pmwa_slot_release.argtypes = [C.c_void_p, C.c_int]
        L.pmwa_slot_progress.argtypes = [C.c_void_p, C.c_int, P(C.c_int64)]
        L.pmwa_chain_status.argtypes = [C.c_void_p, C.c_int]
        L.pmwa_observables.argtypes = [C.c_void_p, C.c_int, P(pmwa_summary)]
        L.pmwa_reset_observables.argtypes = [C.c_void_p]
        L.pmwa_state_hash.argtypes = [C.c_void_p, C.c_int, P(C.c_uint64)]
        L.pmwa_slot_fits.argtypes = [C.c_void_p, C.c_int, P(pmwa_params)]
        L.pmwa_green_static.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_void_p]
        L.pmwa_correlator.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_void_p]
        L.pmwa_worms_general.argtypes = [P(pmwa_localq), C.c_double, C.c_int64, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                         C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_void_p]
        L.pmwa_strerror.argtypes = [C.c_int]
        L.pmwa_strerror.restype = C.c_char_p
        _lib = L
    return _lib


class PmwaError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {lib().pmwa_strerror(code).decode()} ({code})")


def _check(rc, where):
    if rc != 0:
        raise PmwaError(rc, where)


def make_params(**kw) -> pmwa_params:
    d = dict(Lx=4, Ly=4, beta=2.0, t=1.0, V=0.0, mu=0.0, eta=0.1, dom_x=1, dom_y=1,
             dom_tau=1, ticks_log2=24, n_cycle=0, C=math.nan, seed=1, chain_id=0)
    if "L" in kw:
        L = kw.pop("L")
        d["Lx"] = d["Ly"] = L
    d.update(kw)
    p = pmwa_params()
    for k, v in d.items():
        setattr(p, k, v)
    return p


def localq(mats) -> pmwa_localq:
    """Operator types (d x d arrays indexed [out, in]) as a pmwa_localq."""
    g = pmwa_localq()
    g.d = int(mats[0].shape[0])
    g.nalpha = len(mats)
    buf = np.zeros((GQ_AMAX, GQ_DMAX, GQ_DMAX))
    for a, m in enumerate(mats):
        buf[a, :g.d, :g.d] = m
    C.memmove(g.q, buf.ctypes.data, buf.nbytes)
    return g


# --- thin wrappers with the C names -------------------------------------
def pmwa_create(chains, opts=None):
    arr = (pmwa_params * len(chains))(*chains)
    o = opts if opts is not None else pmwa_opts()
    h = C.c_void_p()
    _check(lib().pmwa_create(arr, len(chains), C.byref(o), C.byref(h)), "pmwa_create")
    return h


def pmwa_create_slots(shapes, opts=None):
    arr = (pmwa_params * len(shapes))(*shapes)
    o = opts if opts is not None else pmwa_opts()
    h = C.c_void_p()
    _check(lib().pmwa_create_slots(arr, len(shapes), C.byref(o), C.byref(h)), "pmwa_create_slots")
    return h


def pmwa_slot_load(h, slot, p, target_sweeps):
    _check(lib().pmwa_slot_load(h, slot, C.byref(p), int(target_sweeps)), "pmwa_slot_load")


def pmwa_slot_release(h, slot):
    _check(lib().pmwa_slot_release(h, slot), "pmwa_slot_release")


def pmwa_slot_progress(h, slot):
    n = C.c_int64()
    _check(lib().pmwa_slot_progress(h, slot, C.byref(n)), "pmwa_slot_progress")
    return int(n.value)


def pmwa_sweep(h, n):
    _check(lib().pmwa_sweep(h, int(n)), "pmwa_sweep")


def pmwa_phase(h, phase):
    _check(lib().pmwa_phase(h, int(phase)), "pmwa_phase")


def pmwa_measure(h, chain, max_rows=1 << 22):
    buf = np.zeros(max_rows, dtype=OBS_DTYPE)
    n = C.c_int64()
    rc = lib().pmwa_measure(h, chain, buf.ctypes.data, max_rows, C.byref(n))
    _check(rc, "pmwa_measure")
    return buf[: n.value].copy()


def pmwa_status(h):
    return lib().pmwa_status(h)


def pmwa_get_state(h, chain, n_sites, ntau):
    ne = C.c_int64()
    sw = C.c_uint64()
    _check(lib().pmwa_get_state(h, chain, None, None, None, None, 0, C.byref(ne), C.byref(sw)),
           "pmwa_get_state")
    bstate = np.zeros(n_sites * ntau, np.uint8)
    counts = np.zeros(n_sites * ntau, np.int32)
    ticks = np.zeros(max(ne.value, 1), np.int32)
    infos = np.zeros(max(ne.value, 1), np.uint32)
    _check(lib().pmwa_get_state(h, chain, bstate.ctypes.data, counts.ctypes.data, ticks.ctypes.data,
                                infos.ctypes.data, len(ticks), C.byref(ne), C.byref(sw)),
           "pmwa_get_state")
    return dict(bstate=bstate, counts=counts, ticks=ticks[: ne.value], infos=infos[: ne.value],
                sweep=int(sw.value))


def pmwa_set_state(h, chain, st):
    bstate = np.ascontiguousarray(st["bstate"], np.uint8)
    counts = np.ascontiguousarray(st["counts"], np.int32)
    ticks = np.ascontiguousarray(st["ticks"], np.int32)
    infos = np.ascontiguousarray(st["infos"], np.uint32)
    _check(lib().pmwa_set_state(h, chain, bstate.ctypes.data, counts.ctypes.data, ticks.ctypes.data,
                                infos.ctypes.data, len(ticks), int(st["sweep"])), "pmwa_set_state")


def pmwa_chain_info(h, chain):
    info = pmwa_info()
    _check(lib().pmwa_chain_info(h, chain, C.byref(info)), "pmwa_chain_info")
    return info


def pmwa_default_event_cap(p):
    return lib().pmwa_default_event_cap(C.byref(p))


def pmwa_set_timing(h, enable):
    _check(lib().pmwa_set_timing(h, 1 if enable else 0), "pmwa_set_timing")


def pmwa_set_timing_phases(h, mask):
    _check(lib().pmwa_set_timing_phases(h, int(mask)), "pmwa_set_timing_phases")


def pmwa_phase_times(h):
    ms = np.zeros(7)
    n = np.zeros(7, np.int64)
    _check(lib().pmwa_phase_times(h, ms.ctypes.data, n.ctypes.data), "pmwa_phase_times")
    return ms, n


def pmwa_green(h, chain, disps):
    """Green function G(r, dt) of b + b^+ on the chain's current
    configuration, one value per displacement (rx, ry) or (rx, ry, dt ticks)."""
    rows = [tuple(int(v) for v in dd) + (0,) * (3 - len(dd)) for dd in disps]
    d = np.ascontiguousarray(np.array(rows, dtype=np.int64).reshape(-1, 3), dtype=np.int32)
    out = np.zeros(len(d))
    _check(lib().pmwa_green(h, chain, d.ctypes.data, len(d), out.ctypes.data), "pmwa_green")
    return out


def pmwa_chain_status(h, chain):
    return lib().pmwa_chain_status(h, chain)


def pmwa_observables(h, chain, allow_flagged=False):
    """Accumulated sums and per-site thermal averages of one chain (dict)."""
    out = pmwa_summary()
    rc = lib().pmwa_observables(h, chain, C.byref(out))
    if not allow_flagged:
        _check(rc, "pmwa_observables")
    return {n: getattr(out, n) for n, _ in pmwa_summary._fields_}


def pmwa_reset_observables(h):
    _check(lib().pmwa_reset_observables(h), "pmwa_reset_observables")


def pmwa_state_hash(h, chain):
    v = C.c_uint64()
    _check(lib().pmwa_state_hash(h, chain, C.byref(v)), "pmwa_state_hash")
    return int(v.value)


def pmwa_slot_fits(h, slot, p):
    return lib().pmwa_slot_fits(h, slot, C.byref(p)) == 0


def pmwa_green_static(h, chain, disps):
    """pmwa_green through the entry point that allocates nothing."""
    rows = [tuple(int(v) for v in dd) + (0,) * (3 - len(dd)) for dd in disps]
    d = np.ascontiguousarray(np.array(rows, dtype=np.int64).reshape(-1, 3), dtype=np.int32)
    out = np.zeros(len(d))
    _check(lib().pmwa_green_static(h, chain, d.ctypes.data, len(d), out.ctypes.data), "pmwa_green_static")
    return out


def pmwa_correlator(h, chain, corrs, nbase=8):
    """n-point functions on the current configuration: `corrs` is a list of
    correlators, each a list of points (rx, ry, dt ticks, op), op 0 = b + b^+,
    1 = b, 2 = b^+, all with the same number of points."""
    arr = np.ascontiguousarray(np.array(corrs, dtype=np.int64), dtype=np.int32)
    ncorr, npt = arr.shape[0], arr.shape[1]
    out = np.zeros(ncorr)
    _check(lib().pmwa_correlator(h, chain, npt, arr.ctypes.data, ncorr, nbase, out.ctypes.data), "pmwa_correlator")
    return out


def pmwa_diag(h, chain):
    out = np.zeros(4, np.int64)
    _check(lib().pmwa_diag(h, chain, out.ctypes.data, 4), "pmwa_diag")
    return dict(windows=int(out[0]), windows_max=int(out[1]), attempts=int(out[2]),
                attempts_max=int(out[3]))


def pmwa_destroy(h):
    if h:
        lib().pmwa_destroy(h)


class Sim:
    """A handle of one or more chains (convenience around the calls above)."""

    def __init__(self, chains, stream=None, scatter_mode=0, series_cap=4096, event_cap=0,
                 use_graph=False, regen_mode=0, vertex_mode=0, scatter_lds=0, groups=0, vertex_rows=0):
        if isinstance(chains, pmwa_params):
            chains = [chains]
        self.chains = list(chains)
        o = pmwa_opts()
        o.stream = stream
        o.scatter_mode = scatter_mode
        o.series_cap = series_cap
        o.event_cap = event_cap
        o.use_graph = 1 if use_graph else 0
        o.regen_mode = regen_mode
        o.vertex_mode = vertex_mode
        o.scatter_lds = scatter_lds
        o.groups = groups
        o.vertex_rows = vertex_rows
        self.h = pmwa_create(self.chains, o)

    def close(self):
        if self.h:
            pmwa_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, n=1):
        pmwa_sweep(self.h, n)

    def phase(self, ph):
        pmwa_phase(self.h, ph)

    def measure(self, chain=0):
        return pmwa_measure(self.h, chain)

    def status(self):
        return pmwa_status(self.h)

    def get_state(self, chain=0):
        p = self.chains[chain]
        return pmwa_get_state(self.h, chain, p.Lx * p.Ly, p.dom_tau)

    def set_state(self, st, chain=0):
        pmwa_set_state(self.h, chain, st)

    def info(self, chain=0):
        return pmwa_chain_info(self.h, chain)

    def set_timing(self, enable=True):
        pmwa_set_timing(self.h, enable)

    def set_timing_phases(self, mask):
        """Time only the phases whose bit (phase - 1) is set in `mask`."""
        pmwa_set_timing_phases(self.h, mask)

    def phase_times(self):
        return pmwa_phase_times(self.h)

    def diag(self, chain=0):
        return pmwa_diag(self.h, chain)

    def green(self, disps, chain=0):
        return pmwa_green(self.h, chain, disps)

    def observables(self, chain=0):
        return pmwa_observables(self.h, chain)

    def correlator(self, corrs, nbase=8, chain=0):
        return pmwa_correlator(self.h, chain, corrs, nbase)

    def reset_observables(self):
        pmwa_reset_observables(self.h)

    def state_hash(self, chain=0):
        return pmwa_state_hash(self.h, chain)

    def chain_status(self, chain=0):
        return pmwa_chain_status(self.h, chain)


# --- device buffers through the library's own HIP runtime ---------------
# The general worm law takes device arrays.  They are allocated with the HIP
# runtime that libpmwa.so itself loaded (dlopen by its soname returns that
# copy), so the pointers and streams are those of the library's runtime.
_hip = None
H2D, D2H = 1, 2


def hip():
    global _hip
    if _hip is None:
        lib()
        H = C.CDLL("libamdhip64.so.7")
        H.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        H.hipFree.argtypes = [C.c_void_p]
        H.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        H.hipDeviceSynchronize.argtypes = []
        H.hipStreamCreate.argtypes = [C.POINTER(C.c_void_p)]
        H.hipStreamDestroy.argtypes = [C.c_void_p]
        H.hipStreamSynchronize.argtypes = [C.c_void_p]
        H.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        H.hipEventRecord.argtypes = [C.c_void_p, C.c_void_p]
        H.hipEventSynchronize.argtypes = [C.c_void_p]
        H.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        H.hipEventDestroy.argtypes = [C.c_void_p]
        _hip = H
    return _hip


def _hip_check(rc, where):
    if rc != 0:
        raise PmwaError(PMWA_EDEVICE, f"{where} (hip error {rc})")


class DeviceArray:
    """A device allocation holding one numpy array's worth of data."""

    def __init__(self, shape, dtype):
        self.shape = tuple(shape) if np.ndim(shape) else (int(shape),)
        self.dtype = np.dtype(dtype)
        self.nbytes = int(np.prod(self.shape)) * self.dtype.itemsize
        self.ptr = C.c_void_p()
        _hip_check(hip().hipMalloc(C.byref(self.ptr), max(self.nbytes, 1)), "hipMalloc")

    @classmethod
    def from_numpy(cls, a):
        a = np.ascontiguousarray(a)
        d = cls(a.shape, a.dtype)
        if a.nbytes:
            _hip_check(hip().hipMemcpy(d.ptr, a.ctypes.data, a.nbytes, H2D), "hipMemcpy")
        return d

    def numpy(self):
        a = np.empty(self.shape, self.dtype)
        if self.nbytes:
            _hip_check(hip().hipMemcpy(a.ctypes.data, self.ptr, self.nbytes, D2H), "hipMemcpy")
        return a

    def free(self):
        if self.ptr:
            hip().hipFree(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class DeviceStream:
    """A HIP stream of the library's runtime (default priority)."""

    def __init__(self):
        self.h = C.c_void_p()
        _hip_check(hip().hipStreamCreate(C.byref(self.h)), "hipStreamCreate")

    def synchronize(self):
        _hip_check(hip().hipStreamSynchronize(self.h), "hipStreamSynchronize")

    def close(self):
        if self.h:
            hip().hipStreamDestroy(self.h)
            self.h = C.c_void_p()


class WormsGeneral:
    """Inputs and outputs of pmwa_worms_general for n_int intervals and a
    cap, in device memory: n (int32), slots (int32), alpha, after, dirs
    (uint8), the last four cap x n_int (worm k of interval i at [k, i])."""

    def __init__(self, p, q, ell, cap=64):
        p, q, ell = (np.asarray(a) for a in (p, q, ell))
        self.n_int = int(p.size)
        if q.size != self.n_int or ell.size != self.n_int:
            raise ValueError("p, q and ell must have one length")
        self.cap = int(cap)
        self.p = DeviceArray.from_numpy(p.astype(np.int32))
        self.q = DeviceArray.from_numpy(q.astype(np.int32))
        self.ell = DeviceArray.from_numpy(ell.astype(np.int64))
        self.n = DeviceArray(self.n_int, np.int32)
        k = max(self.cap, 1)
        self.slots = DeviceArray((k, self.n_int), np.int32)
        self.alpha = DeviceArray((k, self.n_int), np.uint8)
        self.after = DeviceArray((k, self.n_int), np.uint8)
        self.dirs = DeviceArray((k, self.n_int), np.uint8)

    def run(self, g, lam, seed=1, stream=0, sweep=0, unit0=0, hip_stream=None):
        """Enqueue the draws (asynchronous on hip_stream, a DeviceStream or
        None for the default stream)."""
        st = hip_stream.h if isinstance(hip_stream, DeviceStream) else hip_stream
        rc = lib().pmwa_worms_general(C.byref(g), float(lam), self.n_int, self.p.ptr, self.q.ptr, self.ell.ptr,
                                      int(seed), int(stream), int(sweep), int(unit0), self.cap, self.n.ptr,
                                      self.slots.ptr, self.alpha.ptr, self.after.ptr, self.dirs.ptr, st)
        _check(rc, "pmwa_worms_general")
        return self

    def result(self):
        """Synchronise the device and copy the outputs to host arrays."""
        _hip_check(hip().hipDeviceSynchronize(), "hipDeviceSynchronize")
        out = dict(n=self.n.numpy())
        for k in ("slots", "alpha", "after", "dirs"):
            out[k] = getattr(self, k).numpy()[:self.cap]
        return out

    def close(self):
        for k in ("p", "q", "ell", "n", "slots", "alpha", "after", "dirs"):
            getattr(self, k).free()


def pmwa_worms_general(g, lam, p, q, ell, seed=1, stream=0, sweep=0, unit0=0, cap=64):
    """Worms of the intervals (p, q, ell host arrays) drawn on the device;
    returns host arrays n, slots, alpha, after, dirs (the last four cap x
    n_int).  See WormsGeneral for device-resident use."""
    w = WormsGeneral(p, q, ell, cap)
    try:
        return w.run(g, lam, seed, stream, sweep, unit0).result()
    finally:
        w.close()
