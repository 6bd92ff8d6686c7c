"""Thin Python binding of the C ABI in include/spkmc.h (argument marshalling only).

Every step of the spkMC cycle runs in the HIP kernels of ``libspkmc.so``;
PyTorch only provides the device buffer and the stream.  Importing this module
fails loudly if the library has not been built (there is no CPU fallback).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspkmc.so")

OK, E_INVAL, E_NOMEM, E_DEVICE, E_STATE, E_RANGE, E_UNSUPPORTED = range(7)
RATES = {"glauber": 0, "metropolis": 1}
INITS = {"random": 0, "up": 1, "down": 2}
LAYOUTS = {"int8": 0, "packed": 1}
ENGINES = {"auto": 0, "cycle": 1, "persistent": 2, "incremental": 3, "slab": 4}
VARIANTS = {"rmax_all": 1, "two_colours": 2, "rmax_bound": 4}


class Params(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("L", C.c_int32), ("domain", C.c_int32), ("rates", C.c_int32),
                ("J", C.c_double), ("H", C.c_double), ("T", C.c_double), ("seed", C.c_uint64),
                ("init", C.c_int32), ("layout", C.c_int32), ("engine", C.c_int32), ("wg_domains", C.c_int32),
                ("record_cap", C.c_uint32), ("variant", C.c_uint32)]


class Record(C.Structure):
    _fields_ = [("cycle", C.c_uint64), ("fired", C.c_uint64), ("nulls", C.c_uint64), ("t", C.c_double),
                ("M", C.c_int64), ("B", C.c_int64)]

    def as_tuple(self):
        return (self.cycle, self.fired, self.nulls, self.t, self.M, self.B)


class Obs(C.Structure):
    _fields_ = [("rec", Record), ("E", C.c_double), ("m", C.c_double), ("ur", C.c_double)]


class Info(C.Structure):
    _fields_ = [("engine", C.c_int32), ("layout", C.c_int32), ("h", C.c_int32), ("grid", C.c_int32),
                ("block", C.c_int32), ("wg_domains", C.c_int32), ("K", C.c_uint64), ("N", C.c_uint64),
                ("state_bytes", C.c_uint64), ("bytes_per_cycle", C.c_double)]


class BatchInfo(C.Structure):
    _fields_ = [("grid", C.c_int32), ("block", C.c_int32), ("wg_domains", C.c_int32), ("h", C.c_int32),
                ("lattices", C.c_uint64), ("domains", C.c_uint64)]


class ServerConfig(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("macro_cycles", C.c_uint32), ("max_live", C.c_uint32),
                ("inflight", C.c_uint32), ("wg_domains", C.c_int32), ("reserved", C.c_uint32)]


class RequestStatus(C.Structure):
    _fields_ = [("state", C.c_int32), ("flags", C.c_uint32), ("ncycles", C.c_uint64),
                ("cycles_enqueued", C.c_uint64), ("bytes", C.c_uint64), ("t_arrival", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("obs", Obs)]


class ServerStats(C.Structure):
    _fields_ = [("queued", C.c_uint64), ("live", C.c_uint64), ("finishing", C.c_uint64), ("done", C.c_uint64),
                ("failed", C.c_uint64), ("macro_steps", C.c_uint64), ("launches", C.c_uint64),
                ("pool_in_use", C.c_uint64), ("pool_peak", C.c_uint64), ("inflight", C.c_uint64)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = range(4)
SERVE_KEEP = 1

EXPORTS = ["spkmc_state_bytes", "spkmc_init", "spkmc_run", "spkmc_observables", "spkmc_records",
           "spkmc_copy_spins", "spkmc_set_spins", "spkmc_rate_table", "spkmc_save", "spkmc_load",
           "spkmc_query", "spkmc_last_error", "spkmc_destroy", "spkmc_batch_workspace_bytes",
           "spkmc_run_batch", "spkmc_run_batch_static", "spkmc_batch_graph_create", "spkmc_batch_graph_launch", "spkmc_batch_graph_destroy",
           "spkmc_server_reserved_bytes", "spkmc_server_create", "spkmc_server_submit",
           "spkmc_server_step", "spkmc_server_poll", "spkmc_server_context", "spkmc_server_release",
           "spkmc_server_clock", "spkmc_server_last_error", "spkmc_server_destroy"]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1005_4713_amd.build` "
                          "(there is no fallback path)")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    P = C.POINTER
    lib.spkmc_state_bytes.restype = C.c_size_t
    lib.spkmc_state_bytes.argtypes = [P(Params)]
    lib.spkmc_init.restype = C.c_int
    lib.spkmc_init.argtypes = [P(Params), vp, C.c_size_t, vp, P(vp)]
    lib.spkmc_run.restype = C.c_int
    lib.spkmc_run.argtypes = [vp, C.c_uint64, C.c_uint32]
    lib.spkmc_observables.restype = C.c_int
    lib.spkmc_observables.argtypes = [vp, P(Obs)]
    lib.spkmc_records.restype = C.c_int
    lib.spkmc_records.argtypes = [vp, P(Record), C.c_size_t, P(C.c_size_t)]
    lib.spkmc_copy_spins.restype = C.c_int
    lib.spkmc_copy_spins.argtypes = [vp, P(C.c_int8), C.c_size_t]
    lib.spkmc_set_spins.restype = C.c_int
    lib.spkmc_set_spins.argtypes = [vp, P(C.c_int8), C.c_size_t]
    lib.spkmc_rate_table.restype = C.c_int
    lib.spkmc_rate_table.argtypes = [P(Params), P(C.c_double)]
    lib.spkmc_save.restype = C.c_int
    lib.spkmc_save.argtypes = [vp, vp, C.c_size_t, P(C.c_size_t)]
    lib.spkmc_load.restype = C.c_int
    lib.spkmc_load.argtypes = [vp, vp, C.c_size_t]
    lib.spkmc_query.restype = C.c_int
    lib.spkmc_query.argtypes = [vp, P(Info)]
    lib.spkmc_last_error.restype = C.c_char_p
    lib.spkmc_last_error.argtypes = [vp]
    lib.spkmc_destroy.restype = None
    lib.spkmc_destroy.argtypes = [vp]
    lib.spkmc_batch_workspace_bytes.restype = C.c_size_t
    lib.spkmc_batch_workspace_bytes.argtypes = [C.c_size_t]
    lib.spkmc_run_batch_static.restype = C.c_int
    lib.spkmc_run_batch_static.argtypes = [P(vp), C.c_size_t, P(C.c_uint64), C.c_uint32, C.c_int32, P(BatchInfo)]
    lib.spkmc_run_batch.restype = C.c_int
    lib.spkmc_run_batch.argtypes = [P(vp), C.c_size_t, P(C.c_uint64), C.c_uint32, C.c_int32, vp, C.c_size_t,
                                    P(BatchInfo)]
    lib.spkmc_batch_graph_create.restype = C.c_int
    lib.spkmc_batch_graph_create.argtypes = [P(vp), C.c_size_t, P(C.c_uint64), C.c_uint32, C.c_int32, vp,
                                             C.c_size_t, P(BatchInfo), P(vp)]
    lib.spkmc_batch_graph_launch.restype = C.c_int
    lib.spkmc_batch_graph_launch.argtypes = [vp, C.c_uint32]
    lib.spkmc_batch_graph_destroy.restype = None
    lib.spkmc_batch_graph_destroy.argtypes = [vp]
    lib.spkmc_server_reserved_bytes.restype = C.c_size_t
    lib.spkmc_server_reserved_bytes.argtypes = [P(ServerConfig)]
    lib.spkmc_server_create.restype = C.c_int
    lib.spkmc_server_create.argtypes = [P(ServerConfig), vp, C.c_size_t, vp, P(vp)]
    lib.spkmc_server_submit.restype = C.c_int
    lib.spkmc_server_submit.argtypes = [vp, P(Params), C.c_uint64, C.c_uint32, C.c_uint32, C.c_double,
                                        P(C.c_uint64)]
    lib.spkmc_server_step.restype = C.c_int
    lib.spkmc_server_step.argtypes = [vp, C.c_int, P(ServerStats)]
    lib.spkmc_server_poll.restype = C.c_int
    lib.spkmc_server_poll.argtypes = [vp, C.c_uint64, P(RequestStatus)]
    lib.spkmc_server_context.restype = C.c_int
    lib.spkmc_server_context.argtypes = [vp, C.c_uint64, P(vp)]
    lib.spkmc_server_release.restype = C.c_int
    lib.spkmc_server_release.argtypes = [vp, C.c_uint64]
    lib.spkmc_server_clock.restype = C.c_double
    lib.spkmc_server_clock.argtypes = [vp]
    lib.spkmc_server_last_error.restype = C.c_char_p
    lib.spkmc_server_last_error.argtypes = [vp]
    lib.spkmc_server_destroy.restype = None
    lib.spkmc_server_destroy.argtypes = [vp]
    return lib


lib = _load()


class SpkmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"spkmc status {status}: {msg}")
        self.status = status


def make_params(L, domain, J=1.0, H=0.0, T=4.5115, seed=1, rates="glauber", init="random",
                layout="packed", engine="auto", wg_domains=0, record_cap=1024, variant=0):
    p = Params()
    p.struct_size = C.sizeof(Params)
    p.L, p.domain = int(L), int(domain)
    p.rates = RATES[rates] if isinstance(rates, str) else int(rates)
    p.J, p.H, p.T = float(J), float(H), float(T)
    p.seed = int(seed)
    p.init = INITS[init] if isinstance(init, str) else int(init)
    p.layout = LAYOUTS[layout] if isinstance(layout, str) else int(layout)
    p.engine = ENGINES[engine] if isinstance(engine, str) else int(engine)
    p.wg_domains = int(wg_domains)
    p.record_cap = int(record_cap)
    if isinstance(variant, str):
        variant = sum(VARIANTS[v] for v in variant.split("|") if v)
    p.variant = int(variant)
    return p


def state_bytes(params):
    return lib.spkmc_state_bytes(C.byref(params))


def rate_table(params):
    out = (C.c_double * 14)()
    st = lib.spkmc_rate_table(C.byref(params), out)
    if st != OK:
        raise SpkmcError(st, lib.spkmc_last_error(None).decode())
    return np.array(list(out))


class _Lattice:
    """Calls on one context (self.ctx, self.params, self.N)."""

    def _check(self, st):
        if st != OK:
            raise SpkmcError(st, lib.spkmc_last_error(self.ctx).decode())

    def run(self, ncycles, obs_every=0):
        self._check(lib.spkmc_run(self.ctx, int(ncycles), int(obs_every)))

    def observables(self):
        o = Obs()
        self._check(lib.spkmc_observables(self.ctx, C.byref(o)))
        return {"cycle": o.rec.cycle, "fired": o.rec.fired, "nulls": o.rec.nulls, "t": o.rec.t,
                "M": o.rec.M, "B": o.rec.B, "E": o.E, "m": o.m, "ur": o.ur}

    def state(self):
        o = Obs()
        self._check(lib.spkmc_observables(self.ctx, C.byref(o)))
        return o.rec.as_tuple()

    def records(self, cap=None):
        cap = self.params.record_cap if cap is None else cap
        buf = (Record * max(cap, 1))()
        n = C.c_size_t()
        self._check(lib.spkmc_records(self.ctx, buf, cap, C.byref(n)))
        return [buf[i].as_tuple() for i in range(n.value)]

    def spins(self):
        out = np.empty(self.N, dtype=np.int8)
        self._check(lib.spkmc_copy_spins(self.ctx, out.ctypes.data_as(C.POINTER(C.c_int8)), out.size))
        return out

    def set_spins(self, spins):
        spins = np.ascontiguousarray(spins, dtype=np.int8)
        self._check(lib.spkmc_set_spins(self.ctx, spins.ctypes.data_as(C.POINTER(C.c_int8)), spins.size))

    def save(self):
        n = C.c_size_t()
        self._check(lib.spkmc_save(self.ctx, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(lib.spkmc_save(self.ctx, buf, n.value, C.byref(n)))
        return buf.raw

    def load(self, blob):
        buf = C.create_string_buffer(blob, len(blob))
        self._check(lib.spkmc_load(self.ctx, buf, len(blob)))

    def info(self):
        i = Info()
        self._check(lib.spkmc_query(self.ctx, C.byref(i)))
        return {f: getattr(i, f) for f, _ in Info._fields_}


class Sim(_Lattice):
    """One lattice on one GPU: the device buffer is a torch uint8 tensor, the
    work runs on torch's current stream of ``device``."""

    def __init__(self, L, domain, device=None, **kw):
        import torch
        self.params = make_params(L, domain, **kw)
        nbytes = state_bytes(self.params)
        if nbytes == 0:
            raise SpkmcError(E_INVAL, lib.spkmc_last_error(None).decode())
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        # 256-byte alignment: the caching allocator returns 512-byte aligned blocks
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            st = lib.spkmc_init(C.byref(self.params), C.c_void_p(self.buf.data_ptr()), nbytes,
                                C.c_void_p(self.stream.cuda_stream), C.byref(self.ctx))
        if st != OK:
            msg = lib.spkmc_last_error(self.ctx if self.ctx else None).decode()
            self._free()
            raise SpkmcError(st, msg)
        self.L = int(L)
        self.N = self.L ** 3

    def _free(self):
        # (at interpreter exit the module's globals may already be gone)
        if getattr(self, "ctx", None) and self.ctx.value and lib is not None:
            lib.spkmc_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        self._free()


_workspace = {}


def release_cached():
    """Wait for the device, then drop the batch workspaces this module keeps
    per stream, so that a program can free every device buffer of the library
    before the interpreter and the HIP runtime shut down (each Sim, Server or
    BatchGraph is released by dropping it, or by its close())."""
    if _workspace:
        import torch
        torch.cuda.synchronize()
        _workspace.clear()


def run_batch(sims, ncycles, obs_every=0, wg_domains=0):
    """Run ncycles[i] cycles on each lattice of `sims` (same device, stream and
    octant edge) in one persistent launch; returns the launch shape."""
    import torch
    n = len(sims)
    if n == 0:
        return None
    if isinstance(ncycles, int):
        ncycles = [ncycles] * n
    need = lib.spkmc_batch_workspace_bytes(n)
    dev = sims[0].device
    # one workspace per stream: launches on one stream run in order, so the next
    # batch's descriptors never overwrite those of a batch still running
    key = (str(dev), sims[0].stream.cuda_stream)
    ws = _workspace.get(key)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1 << 16), dtype=torch.uint8, device=dev)
        _workspace[key] = ws
    ctxs = (C.c_void_p * n)(*[sim.ctx.value for sim in sims])
    cyc = (C.c_uint64 * n)(*[int(c) for c in ncycles])
    info = BatchInfo()
    st = lib.spkmc_run_batch(ctxs, n, cyc, int(obs_every), int(wg_domains), C.c_void_p(ws.data_ptr()),
                             ws.numel(), C.byref(info))
    if st != OK:
        raise SpkmcError(st, lib.spkmc_last_error(None).decode())
    return {f: getattr(info, f) for f, _ in BatchInfo._fields_}


def run_batch_static(sims, ncycles, obs_every=0, wg_domains=0):
    """run_batch without a workspace: the descriptors go into the library's own
    device array (at most 512 lattices; no device allocation)."""
    n = len(sims)
    if n == 0:
        return None
    if isinstance(ncycles, int):
        ncycles = [ncycles] * n
    ctxs = (C.c_void_p * n)(*[sim.ctx.value for sim in sims])
    cyc = (C.c_uint64 * n)(*[int(c) for c in ncycles])
    info = BatchInfo()
    st = lib.spkmc_run_batch_static(ctxs, n, cyc, int(obs_every), int(wg_domains), C.byref(info))
    if st != OK:
        raise SpkmcError(st, lib.spkmc_last_error(None).decode())
    return {f: getattr(info, f) for f, _ in BatchInfo._fields_}


class BatchGraph:
    """One batch macro-step (ncycles[i] cycles of each lattice) captured into a
    HIP graph by the library and replayed with launch(replays); the graph owns
    its own descriptor workspace (see spkmc_batch_graph_*)."""

    def __init__(self, sims, ncycles, obs_every=0, wg_domains=0):
        import torch
        n = len(sims)
        if isinstance(ncycles, int):
            ncycles = [ncycles] * n
        self.sims = list(sims)  # the lattices stay alive with the graph
        self.ws = torch.empty(max(lib.spkmc_batch_workspace_bytes(n), 1 << 16), dtype=torch.uint8,
                              device=sims[0].device)
        ctxs = (C.c_void_p * n)(*[sim.ctx.value for sim in sims])
        cyc = (C.c_uint64 * n)(*[int(c) for c in ncycles])
        info = BatchInfo()
        self.g = C.c_void_p()
        st = lib.spkmc_batch_graph_create(ctxs, n, cyc, int(obs_every), int(wg_domains),
                                          C.c_void_p(self.ws.data_ptr()), self.ws.numel(), C.byref(info),
                                          C.byref(self.g))
        if st != OK:
            raise SpkmcError(st, lib.spkmc_last_error(None).decode())
        self.info = {f: getattr(info, f) for f, _ in BatchInfo._fields_}

    def launch(self, replays=1):
        st = lib.spkmc_batch_graph_launch(self.g, int(replays))
        if st != OK:
            raise SpkmcError(st, lib.spkmc_last_error(None).decode())

    def close(self):
        if getattr(self, "g", None) and lib is not None:
            import torch
            torch.cuda.synchronize(self.ws.device)  # the last replay reads the workspace
            lib.spkmc_batch_graph_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The request server of the library over a torch device pool and torch's
    current stream: continuous batching of whole lattices (see spkmc_server_*)."""

    def __init__(self, pool_bytes, macro_cycles=100, max_live=512, inflight=2, wg_domains=0, device=None):
        import torch
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        cfg = ServerConfig()
        cfg.struct_size = C.sizeof(ServerConfig)
        cfg.macro_cycles, cfg.max_live, cfg.inflight = int(macro_cycles), int(max_live), int(inflight)
        cfg.wg_domains, cfg.reserved = int(wg_domains), 0
        self.cfg = cfg
        self.reserved = lib.spkmc_server_reserved_bytes(C.byref(cfg))
        if self.reserved == 0:
            raise SpkmcError(E_INVAL, "invalid server configuration")
        self.pool = torch.empty(int(pool_bytes) + self.reserved, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.h = C.c_void_p()
        with torch.cuda.device(self.device):
            st = lib.spkmc_server_create(C.byref(cfg), C.c_void_p(self.pool.data_ptr()), self.pool.numel(),
                                         C.c_void_p(self.stream.cuda_stream), C.byref(self.h))
        if st != OK:
            raise SpkmcError(st, lib.spkmc_server_last_error(None).decode())

    def _check(self, st):
        if st != OK:
            raise SpkmcError(st, lib.spkmc_server_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) and self.h.value and lib is not None:
            lib.spkmc_server_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        self.close()

    def submit(self, L, domain, ncycles, obs_every=0, keep=False, t_arrival=-1.0, **kw):
        p = make_params(L, domain, **kw)
        rid = C.c_uint64()
        self._check(lib.spkmc_server_submit(self.h, C.byref(p), int(ncycles), int(obs_every),
                                            SERVE_KEEP if keep else 0, float(t_arrival), C.byref(rid)))
        return rid.value

    def step(self, wait=False):
        s = ServerStats()
        self._check(lib.spkmc_server_step(self.h, 1 if wait else 0, C.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def poll(self, rid):
        r = RequestStatus()
        self._check(lib.spkmc_server_poll(self.h, int(rid), C.byref(r)))
        out = {f: getattr(r, f) for f, _ in RequestStatus._fields_ if f != "obs"}
        out["state_tuple"] = r.obs.rec.as_tuple()
        out["E"], out["m"], out["ur"] = r.obs.E, r.obs.m, r.obs.ur
        return out

    def lattice(self, rid, L, record_cap=1024):
        """The kept lattice of a DONE request (valid until release)."""
        ctx = C.c_void_p()
        self._check(lib.spkmc_server_context(self.h, int(rid), C.byref(ctx)))
        v = _Lattice()
        v.ctx, v.N = ctx, int(L) ** 3
        v.params = make_params(L, 2, record_cap=record_cap)
        return v

    def release(self, rid):
        self._check(lib.spkmc_server_release(self.h, int(rid)))

    def clock(self):
        return lib.spkmc_server_clock(self.h)

    def drain(self, wait=True):
        """Step until nothing is queued, resident or in flight."""
        while True:
            st = self.step(wait=wait)
            if st["queued"] == 0 and st["live"] == 0 and st["inflight"] == 0:
                return st
