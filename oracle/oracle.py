"""ctypes binding of the C oracle (test infrastructure only)."""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle_spkmc.so")


class Params(C.Structure):
    _fields_ = [("L", C.c_int32), ("d", C.c_int32), ("J", C.c_double), ("H", C.c_double),
                ("T", C.c_double), ("seed", C.c_uint64), ("rates", C.c_int32), ("init", C.c_int32),
                ("colours", C.c_int32), ("rmax_scope", C.c_int32), ("order", C.c_int32),
                ("check", C.c_int32)]


class Record(C.Structure):
    _fields_ = [("cycle", C.c_uint64), ("fired", C.c_uint64), ("nulls", C.c_uint64),
                ("t", C.c_double), ("M", C.c_int64), ("B", C.c_int64)]

    def as_tuple(self):
        return (self.cycle, self.fired, self.nulls, self.t, self.M, self.B)


def _load():
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(LIB_PATH)
    u32p = C.POINTER(C.c_uint32)
    f64p = C.POINTER(C.c_double)
    i64p = C.POINTER(C.c_int64)
    i8p = C.POINTER(C.c_int8)
    vp = C.c_void_p
    sigs = {
        "orc_philox4x32_10": (None, [u32p, u32p, u32p]),
        "orc_u53": (C.c_double, [C.c_uint32, C.c_uint32]),
        "orc_uopen52": (C.c_double, [C.c_uint32, C.c_uint32]),
        "orc_idx": (C.c_uint32, [C.c_uint32, C.c_uint32]),
        "orc_rate_table": (C.c_int, [C.c_double, C.c_double, C.c_double, C.c_int32, f64p]),
        "orc_select": (C.c_int, [u32p, f64p, C.c_double, C.c_double, C.c_uint32,
                                 C.POINTER(C.c_int32), u32p]),
        "orc_sim_new": (vp, [C.POINTER(Params)]),
        "orc_sim_free": (None, [vp]),
        "orc_sim_run": (C.c_int, [vp, C.c_uint64, C.c_uint32, C.POINTER(Record), C.c_uint64,
                                  C.POINTER(C.c_uint64)]),
        "orc_sim_state": (None, [vp, C.POINTER(Record)]),
        "orc_sim_check_failures": (C.c_uint64, [vp]),
        "orc_sim_get_spins": (None, [vp, i8p]),
        "orc_sim_rate": (C.c_double, [vp, C.c_int]),
        "orc_sim_rbound": (C.c_double, [vp]),
        "orc_sim_set_state": (C.c_int, [vp, i8p, C.c_uint64, C.c_uint64, C.c_uint64, C.c_double]),
        "orc_sim_octant_hist": (None, [vp, C.c_uint32, C.c_int32, u32p]),
        "orc_sim_run_grid": (C.c_uint64, [vp, f64p, C.c_uint64, i64p, i64p, C.c_uint64]),
        "orc_sim_run_tw": (None, [vp, C.c_uint64, f64p, f64p]),
        "orc_bkl_new": (vp, [C.POINTER(Params), C.c_int32, C.c_int32]),
        "orc_bkl_free": (None, [vp]),
        "orc_bkl_run": (None, [vp, C.c_uint64]),
        "orc_bkl_state": (None, [vp, C.POINTER(Record)]),
        "orc_bkl_get_spins": (None, [vp, i8p]),
        "orc_bkl_counts": (None, [vp, u32p]),
        "orc_bkl_run_grid": (C.c_uint64, [vp, f64p, C.c_uint64, i64p, i64p, C.c_uint64]),
        "orc_bkl_run_tw": (None, [vp, C.c_uint64, f64p, f64p]),
        "orc_observables": (None, [i8p, C.c_int32, i64p, i64p]),
        "orc_site_class": (C.c_int32, [i8p, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
        "orc_init_spins": (None, [i8p, C.c_int64, C.c_uint64, C.c_int32]),
        "orc_set_threads": (None, [C.c_int32]),
        "orc_get_threads": (C.c_int32, []),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _p(arr, ctype):
    return arr.ctypes.data_as(C.POINTER(ctype))


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib.orc_philox4x32_10(c, k, o)
    return tuple(o)


def u53(a, b):
    return lib.orc_u53(a, b)


def uopen52(a, b):
    return lib.orc_uopen52(a, b)


def idx(w, n):
    return lib.orc_idx(w, n)


def rate_table(J, H, T, rates=0):
    out = (C.c_double * 14)()
    rc = lib.orc_rate_table(J, H, T, rates, out)
    if rc != 0:
        raise ValueError(f"invalid rate parameters (code {rc})")
    return np.array(list(out), dtype=np.float64)


def select(hist, r, Rmax, u, w):
    h = (C.c_uint32 * 14)(*[int(v) for v in hist])
    rr = (C.c_double * 14)(*[float(v) for v in r])
    c = C.c_int32()
    j = C.c_uint32()
    fire = lib.orc_select(h, rr, Rmax, u, w, C.byref(c), C.byref(j))
    return (c.value, j.value) if fire else None


def observables(spins):
    spins = np.ascontiguousarray(spins, dtype=np.int8)
    L = round(spins.size ** (1 / 3))
    M = C.c_int64()
    B = C.c_int64()
    lib.orc_observables(_p(spins, C.c_int8), L, C.byref(M), C.byref(B))
    return M.value, B.value


def site_class(spins, x, y, z):
    spins = np.ascontiguousarray(spins, dtype=np.int8)
    L = round(spins.size ** (1 / 3))
    return lib.orc_site_class(_p(spins, C.c_int8), L, x, y, z)


def init_spins(L, seed, init=0):
    out = np.empty(L ** 3, dtype=np.int8)
    lib.orc_init_spins(_p(out, C.c_int8), L ** 3, seed, init)
    return out


def set_threads(n):
    """Threads of the per-domain loops of a cycle (1 = the plain serial loops;
    any count gives the same trajectory bit for bit)."""
    lib.orc_set_threads(int(n))


def get_threads():
    return lib.orc_get_threads()


def make_params(L, d, J=1.0, H=0.0, T=4.5115, seed=1, rates=0, init=0, colours=8,
                rmax_scope=0, order=0, check=0):
    return Params(L, d, J, H, T, seed, rates, init, colours, rmax_scope, order, check)


class Sim:
    """The plain spkMC simulator (int8 spins, nested loops)."""

    def __init__(self, **kw):
        self.params = make_params(**kw)
        self.L = self.params.L
        self.N = self.L ** 3
        self.h = lib.orc_sim_new(C.byref(self.params))
        if not self.h:
            raise ValueError("invalid oracle parameters")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib.orc_sim_free(h)
            self.h = None

    def run(self, ncycles, obs_every=0):
        cap = ncycles // obs_every + 1 if obs_every else 0
        recs = (Record * max(cap, 1))()
        n = C.c_uint64()
        lib.orc_sim_run(self.h, ncycles, obs_every, recs, cap, C.byref(n))
        return [recs[i].as_tuple() for i in range(min(n.value, cap))]

    def state(self):
        r = Record()
        lib.orc_sim_state(self.h, C.byref(r))
        return r.as_tuple()

    def spins(self):
        out = np.empty(self.N, dtype=np.int8)
        lib.orc_sim_get_spins(self.h, _p(out, C.c_int8))
        return out

    def set_state(self, spins, cycle=0, fired=0, nulls=0, t=0.0):
        spins = np.ascontiguousarray(spins, dtype=np.int8)
        if lib.orc_sim_set_state(self.h, _p(spins, C.c_int8), cycle, fired, nulls, t) != 0:
            raise ValueError("spins must be +-1")

    def check_failures(self):
        return lib.orc_sim_check_failures(self.h)

    def octant_hist(self, k, s):
        out = (C.c_uint32 * 14)()
        lib.orc_sim_octant_hist(self.h, k, s, out)
        return list(out)

    def rates(self):
        return np.array([lib.orc_sim_rate(self.h, c) for c in range(14)])

    def rbound(self):
        return lib.orc_sim_rbound(self.h)

    def run_grid(self, grid, max_cycles=1 << 62):
        grid = np.ascontiguousarray(grid, dtype=np.float64)
        M = np.zeros(grid.size, dtype=np.int64)
        B = np.zeros(grid.size, dtype=np.int64)
        n = lib.orc_sim_run_grid(self.h, _p(grid, C.c_double), grid.size, _p(M, C.c_int64),
                                 _p(B, C.c_int64), max_cycles)
        return M[:n], B[:n]

    def run_tw(self, ncycles, state_hist=False):
        tw = np.zeros(4, dtype=np.float64)
        hist = np.zeros(1 << self.N, dtype=np.float64) if state_hist and self.N <= 16 else None
        lib.orc_sim_run_tw(self.h, ncycles, _p(tw, C.c_double),
                           _p(hist, C.c_double) if hist is not None else None)
        return tw, hist


class Bkl:
    """The serial rejection-free (BKL / n-fold way) simulator."""

    def __init__(self, canonical=0, draw_mode=0, **kw):
        self.params = make_params(**{"d": kw.pop("d", 2), **kw})
        self.L = self.params.L
        self.N = self.L ** 3
        self.h = lib.orc_bkl_new(C.byref(self.params), canonical, draw_mode)
        if not self.h:
            raise ValueError("invalid oracle parameters")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib.orc_bkl_free(h)
            self.h = None

    def run(self, nevents):
        lib.orc_bkl_run(self.h, nevents)

    def state(self):
        r = Record()
        lib.orc_bkl_state(self.h, C.byref(r))
        return r.as_tuple()

    def spins(self):
        out = np.empty(self.N, dtype=np.int8)
        lib.orc_bkl_get_spins(self.h, _p(out, C.c_int8))
        return out

    def counts(self):
        out = (C.c_uint32 * 14)()
        lib.orc_bkl_counts(self.h, out)
        return list(out)

    def run_grid(self, grid, max_events=1 << 62):
        grid = np.ascontiguousarray(grid, dtype=np.float64)
        M = np.zeros(grid.size, dtype=np.int64)
        B = np.zeros(grid.size, dtype=np.int64)
        n = lib.orc_bkl_run_grid(self.h, _p(grid, C.c_double), grid.size, _p(M, C.c_int64),
                                 _p(B, C.c_int64), max_events)
        return M[:n], B[:n]

    def run_tw(self, nevents, state_hist=False):
        tw = np.zeros(4, dtype=np.float64)
        hist = np.zeros(1 << self.N, dtype=np.float64) if state_hist and self.N <= 16 else None
        lib.orc_bkl_run_tw(self.h, nevents, _p(tw, C.c_double),
                           _p(hist, C.c_double) if hist is not None else None)
        return tw, hist
