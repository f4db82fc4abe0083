"""ctypes binding of the serial CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the CPU-baseline leg of
the benchmark use this module; the GPU library never imports it.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "pmwa_oracle.c")

PH_V, PH_R, PH_S, PH_BT, PH_BSX, PH_BSY, PH_END = 1, 2, 3, 4, 5, 6, 7
RNG_V, RNG_R, RNG_S, RNG_BT, RNG_BS = 1, 2, 3, 4, 5


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2 -ffp-contract=off)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Params(C.Structure):
    _fields_ = [("Lx", C.c_int32), ("Ly", C.c_int32), ("beta", C.c_double),
                ("t", C.c_double), ("V", C.c_double), ("mu", C.c_double), ("eta", C.c_double),
                ("dom_x", C.c_int32), ("dom_y", C.c_int32), ("dom_tau", C.c_int32),
                ("ticks_log2", C.c_int32), ("n_cycle", C.c_int32), ("C", C.c_double),
                ("seed", C.c_uint64), ("chain_id", C.c_uint32), ("pad_", C.c_uint32)]


class Obs(C.Structure):
    _fields_ = [("nv", C.c_int64), ("nkink", C.c_int64), ("nw", C.c_int64),
                ("occ2", C.c_int64), ("nn2", C.c_int64), ("qimp", C.c_double)]


class Derived(C.Structure):
    _fields_ = [("C", C.c_double), ("rho_max", C.c_double), ("lam", C.c_double),
                ("delta", C.c_double), ("wd", C.c_double * 4), ("acc", C.c_double * 4),
                ("n_cycle", C.c_int32), ("M", C.c_int32), ("ntau", C.c_int32),
                ("T", C.c_int32 * 65)]


class Summary(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("sweeps", "nv", "nkink", "nw", "occ2", "nn2")] + \
               [(n, C.c_double) for n in ("qimp", "nv_sq", "nkink_sq", "nw_sq", "occ2_sq", "nn2_sq",
                                          "qimp_sq", "E", "E_alt", "E_eta", "density", "Q", "Q_imp",
                                          "b", "err_E", "err_density", "err_Q", "err_Q_imp")]


GQ_DMAX, GQ_AMAX, GQ_CAPMAX = 8, 4, 255
ORC_ECAP = -4


class LocalQ(C.Structure):
    _fields_ = [("d", C.c_int32), ("nalpha", C.c_int32),
                ("q", C.c_double * (GQ_AMAX * GQ_DMAX * GQ_DMAX))]


OBS_DTYPE = np.dtype([("nv", "<i8"), ("nkink", "<i8"), ("nw", "<i8"),
                      ("occ2", "<i8"), ("nn2", "<i8"), ("qimp", "<f8")])

_lib = None


def bind(path: str):
    """Load an oracle library built from pmwa_oracle.c and declare its
    signatures (lib() uses this for the in-tree build)."""
    L = C.CDLL(path)
    P = C.POINTER
    L.orc_create.argtypes = [P(Params), P(C.c_void_p)]
    L.orc_destroy.argtypes = [C.c_void_p]
    L.orc_sweep.argtypes = [C.c_void_p, C.c_int64]
    L.orc_phase.argtypes = [C.c_void_p, C.c_int]
    L.orc_series.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
    L.orc_series.restype = C.c_int64
    L.orc_flags.argtypes = [C.c_void_p]
    L.orc_state_events.argtypes = [C.c_void_p]
    L.orc_state_events.restype = C.c_int64
    L.orc_get_state.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_int64, P(C.c_uint64)]
    L.orc_set_state.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_int64, C.c_uint64]
    L.orc_check.argtypes = [C.c_void_p]
    L.orc_get_derived.argtypes = [C.c_void_p, P(Derived)]
    L.orc_get_scatter_table.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_vertex_weight.argtypes = [C.c_void_p, C.c_int]
    L.orc_vertex_weight.restype = C.c_double
    L.orc_fleg.argtypes = [C.c_void_p, C.c_int, C.c_int64]
    L.orc_fleg.restype = C.c_double
    L.orc_tanh_ell.argtypes = [C.c_void_p, C.c_int64]
    L.orc_tanh_ell.restype = C.c_double
    L.orc_poisson_table.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int]
    L.orc_test_worms.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_int32, C.c_int,
                                 C.c_void_p, C.c_void_p, C.c_int]
    L.orc_test_choose.argtypes = [C.c_void_p, C.c_int, C.c_double]
    L.orc_test_temporal_p0.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int64, C.c_int64]
    L.orc_test_temporal_p0.restype = C.c_double
    L.orc_philox.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_stream_word.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint64]
    L.orc_stream_word.restype = C.c_uint64
    L.orc_green.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
    L.orc_correlator.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_void_p]
    L.orc_observables.argtypes = [C.c_void_p, P(Summary)]
    L.orc_reset_observables.argtypes = [C.c_void_p]
    L.orc_reset_observables.restype = None
    L.orc_state_hash.argtypes = [C.c_void_p]
    L.orc_state_hash.restype = C.c_uint64
    L.orc_worms_general.argtypes = [P(LocalQ), C.c_double, C.c_int64, C.c_int, C.c_int, C.c_uint64,
                                    C.c_uint32, C.c_uint32, C.c_uint32, C.c_int, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p]
    return L


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = bind(LIB_PATH)
    return _lib


def compile_variant(src_text: str, out_path: str) -> str:
    """Compile a (modified) copy of the oracle source to `out_path`, with the
    flags of build(); tests use it to check that a pin catches a planted
    mistake."""
    c_path = out_path[:-3] + ".c" if out_path.endswith(".so") else out_path + ".c"
    with open(c_path, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-w",
                           "-I", HERE, "-o", out_path, c_path, "-lm"])
    return out_path


def make_params(**kw) -> Params:
    d = dict(Lx=4, Ly=4, beta=2.0, t=1.0, V=0.0, mu=0.0, eta=0.1, dom_x=1, dom_y=1,
             dom_tau=1, ticks_log2=24, n_cycle=0, C=math.nan, seed=1, chain_id=0)
    if "L" in kw:
        L = kw.pop("L")
        d["Lx"] = d["Ly"] = L
    d.update(kw)
    p = Params()
    for k, v in d.items():
        setattr(p, k, v)
    return p


def local_q(mats) -> LocalQ:
    """Pack operator types (d x d arrays, [out, in]) into the oracle's struct."""
    g = LocalQ()
    g.d = int(mats[0].shape[0])
    g.nalpha = len(mats)
    buf = np.zeros((GQ_AMAX, GQ_DMAX, GQ_DMAX))
    for a, m in enumerate(mats):
        buf[a, :g.d, :g.d] = m
    C.memmove(g.q, buf.ctypes.data, buf.nbytes)
    return g


def worms_general(g: LocalQ, lam, ell, p, q, seed=1, stream=0, sweep=0, unit=0, cap=GQ_CAPMAX,
                  library=None):
    """Worms of one interval for a general local operator (orc_worms_general):
    returns (n, slots, alpha, after, dirs); n < 0 is the error code."""
    L = library if library is not None else lib()
    slots = np.zeros(max(cap, 1), dtype=np.int32)
    alpha = np.zeros(max(cap, 1), dtype=np.uint8)
    after = np.zeros(max(cap, 1), dtype=np.uint8)
    dirs = np.zeros(max(cap, 1), dtype=np.uint8)
    n = L.orc_worms_general(C.byref(g), float(lam), int(ell), int(p), int(q), int(seed), int(stream),
                            int(sweep), int(unit), int(cap), slots.ctypes.data, alpha.ctypes.data,
                            after.ctypes.data, dirs.ctypes.data)
    k = max(n, 0)
    return n, slots[:k], alpha[:k], after[:k], dirs[:k]


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox(c, k, o)
    return [int(x) for x in o]


class Chain:
    """One oracle chain; mirrors the C-ABI calls of the GPU library."""

    def __init__(self, params: Params | None = None, library=None, **kw):
        self.params = params if params is not None else make_params(**kw)
        self._L = library if library is not None else lib()
        h = C.c_void_p()
        rc = self._L.orc_create(C.byref(self.params), C.byref(h))
        if rc != 0:
            raise ValueError(f"orc_create failed ({rc})")
        self.h = h
        self.N = self.params.Lx * self.params.Ly
        self.ntau = self.params.dom_tau

    def close(self):
        if self.h:
            self._L.orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, n=1):
        rc = self._L.orc_sweep(self.h, n)
        if rc != 0:
            raise RuntimeError(f"orc_sweep failed ({rc}), flags={self.flags()}")

    def phase(self, ph):
        rc = self._L.orc_phase(self.h, ph)
        if rc != 0:
            raise RuntimeError(f"orc_phase({ph}) failed ({rc}), flags={self.flags()}")

    def flags(self):
        return self._L.orc_flags(self.h)

    def check(self):
        return self._L.orc_check(self.h)

    def series(self, max_rows=1 << 30):
        n_total = max_rows
        out = np.zeros(0, dtype=OBS_DTYPE)
        chunks = []
        while n_total > 0:
            buf = np.zeros(min(n_total, 1 << 16), dtype=OBS_DTYPE)
            n = self._L.orc_series(self.h, buf.ctypes.data, len(buf))
            if n <= 0:
                break
            chunks.append(buf[:n])
            n_total -= n
            if n < len(buf):
                break
        return np.concatenate(chunks) if chunks else out

    def get_state(self):
        ne = self._L.orc_state_events(self.h)
        bstate = np.zeros(self.N * self.ntau, np.uint8)
        counts = np.zeros(self.N * self.ntau, np.int32)
        ticks = np.zeros(max(ne, 1), np.int32)
        infos = np.zeros(max(ne, 1), np.uint32)
        sw = C.c_uint64()
        rc = self._L.orc_get_state(self.h, bstate.ctypes.data, counts.ctypes.data,
                                 ticks.ctypes.data, infos.ctypes.data, ne, C.byref(sw))
        if rc != 0:
            raise RuntimeError("orc_get_state failed")
        return dict(bstate=bstate, counts=counts, ticks=ticks[:ne], infos=infos[:ne],
                    sweep=int(sw.value))

    def set_state(self, st):
        bstate = np.ascontiguousarray(st["bstate"], np.uint8)
        counts = np.ascontiguousarray(st["counts"], np.int32)
        ticks = np.ascontiguousarray(st["ticks"], np.int32)
        infos = np.ascontiguousarray(st["infos"], np.uint32)
        rc = self._L.orc_set_state(self.h, bstate.ctypes.data, counts.ctypes.data,
                                 ticks.ctypes.data, infos.ctypes.data, len(ticks),
                                 int(st["sweep"]))
        if rc != 0:
            raise RuntimeError("orc_set_state failed")

    def derived(self):
        d = Derived()
        self._L.orc_get_derived(self.h, C.byref(d))
        return d

    def scatter_table(self):
        tab = np.zeros((16, 4, 4))
        pair = np.zeros((16, 4, 4))
        self._L.orc_get_scatter_table(self.h, tab.ctypes.data, pair.ctypes.data)
        return tab, pair

    def vertex_weight(self, S):
        return self._L.orc_vertex_weight(self.h, S)

    def fleg(self, sigma, ell):
        return self._L.orc_fleg(self.h, sigma, ell)

    def tanh_ell(self, ell):
        return self._L.orc_tanh_ell(self.h, ell)

    def poisson_table(self, k=0):
        buf = np.zeros(1024)
        n = self._L.orc_poisson_table(self.h, k, buf.ctypes.data, 1024)
        return buf[:n]

    def sample_worms(self, unit, ell, sigma, phase=RNG_R):
        off = np.zeros(4096, np.int32)
        dirs = np.zeros(4096, np.uint8)
        n = self._L.orc_test_worms(self.h, phase, unit, ell, sigma, off.ctypes.data,
                                 dirs.ctypes.data, 4096)
        return off[:n].copy(), dirs[:n].copy()

    def temporal_p0(self, p, q, l1, l2):
        return self._L.orc_test_temporal_p0(self.h, p, q, l1, l2)

    def green(self, disps):
        """Green function G(r, dt) of b + b^+ on the current configuration,
        for each displacement (rx, ry) or (rx, ry, dt ticks) in `disps`."""
        rows = [tuple(int(v) for v in dd) + (0,) * (3 - len(dd)) for dd in disps]
        d = np.ascontiguousarray(np.array(rows, dtype=np.int64).reshape(-1, 3), dtype=np.int32)
        out = np.zeros(len(d))
        if self._L.orc_green(self.h, d.ctypes.data, len(d), out.ctypes.data) != 0:
            raise RuntimeError("orc_green failed")
        return out

    def correlator(self, corrs, nbase=8):
        """n-point functions on the current configuration: `corrs` is a list
        of correlators, each a list of points (rx, ry, dt ticks, op) with op
        0 = b + b^+, 1 = b, 2 = b^+ (all correlators with the same number of
        points); one value per correlator."""
        arr = np.ascontiguousarray(np.array(corrs, dtype=np.int64), dtype=np.int32)
        ncorr, npt = arr.shape[0], arr.shape[1]
        out = np.zeros(ncorr)
        if self._L.orc_correlator(self.h, npt, arr.ctypes.data, ncorr, nbase, out.ctypes.data) != 0:
            raise RuntimeError("orc_correlator failed")
        return out

    def observables(self):
        """Accumulated sums and the per-site thermal averages (dict)."""
        out = Summary()
        self._L.orc_observables(self.h, C.byref(out))
        return {n: getattr(out, n) for n, _ in Summary._fields_}

    def reset_observables(self):
        self._L.orc_reset_observables(self.h)

    def state_hash(self):
        return int(self._L.orc_state_hash(self.h))

    def stream_word(self, phase, unit, w):
        return int(self._L.orc_stream_word(self.h, phase, unit, w))


def choose(weights, u):
    w = np.ascontiguousarray(weights, np.float64)
    return lib().orc_test_choose(w.ctypes.data, len(w), u)
