"""The C ABI without a GPU: the library loads, exports every entry point that
include/spkmc.h declares, validates parameters and computes the same FP64 rate
table as the oracle bit for bit."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1005_4713_amd", "libspkmc.so")


@pytest.fixture(scope="module")
def spkmc():
    if not os.path.exists(LIB):
        from paper_1005_4713_amd import build
        build.build()
    from paper_1005_4713_amd import spkmc as mod
    return mod


def _declared():
    src = open(os.path.join(ROOT, "include", "spkmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spkmc_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(spkmc):
    names = _declared()
    assert len(names) >= 13
    lib = C.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(spkmc.EXPORTS) == names


def test_struct_sizes_match_header(spkmc):
    # field layout of the ctypes mirrors: 72-byte params, 48-byte record
    assert C.sizeof(spkmc.Params) == 72
    assert C.sizeof(spkmc.Record) == 48
    assert C.sizeof(spkmc.Obs) == 72


@pytest.mark.parametrize("kw", [dict(L=16, domain=3), dict(L=16, domain=6), dict(L=1, domain=2),
                                dict(L=16, domain=8, T=0.0), dict(L=16, domain=8, T=-1.0),
                                dict(L=16, domain=8, T=1e-3), dict(L=12, domain=6, layout="packed"),
                                dict(L=16, domain=4, layout="packed"), dict(L=16, domain=8, rates=7),
                                dict(L=16, domain=8, init=5), dict(L=16, domain=8, engine=9),
                                dict(L=8192, domain=32, layout="packed"),       # L above 4096
                                dict(L=4096, domain=2),                         # 2^33 lines
                                dict(L=2048, domain=2, variant=2),              # 2^32 lines (two colours)
                                dict(L=4096, domain=4096),                      # octant of 2^33 sites
                                dict(L=4096, domain=4096, layout="packed")])
def test_invalid_parameters(spkmc, kw):
    p = spkmc.make_params(**kw)
    assert spkmc.state_bytes(p) == 0
    assert spkmc.lib.spkmc_last_error(None)
    with pytest.raises(spkmc.SpkmcError):
        spkmc.rate_table(p)
    ctx = C.c_void_p()
    st = spkmc.lib.spkmc_init(C.byref(p), None, 0, None, C.byref(ctx))
    assert st == spkmc.E_INVAL
    spkmc.lib.spkmc_destroy(ctx)


def test_struct_size_checked(spkmc):
    p = spkmc.make_params(16, 8)
    p.struct_size = 64
    assert spkmc.state_bytes(p) == 0
    for bad in (8, 16, 1 | 4, 1 | 2 | 4):  # unknown bits; RMAX_ALL with RMAX_BOUND
        p = spkmc.make_params(16, 8)
        p.variant = bad
        assert spkmc.state_bytes(p) == 0, bad
    for ok in (0, 1, 2, 4, 1 | 2, 2 | 4):
        assert spkmc.state_bytes(spkmc.make_params(16, 8, variant=ok)) > 0, ok


def test_buffer_too_small_rejected(spkmc):
    p = spkmc.make_params(16, 8, layout="int8")
    need = spkmc.state_bytes(p)
    assert need > 16 ** 3
    ctx = C.c_void_p()
    st = spkmc.lib.spkmc_init(C.byref(p), C.c_void_p(1 << 20), need - 1, None, C.byref(ctx))
    assert st == spkmc.E_RANGE
    spkmc.lib.spkmc_destroy(ctx)


@pytest.mark.parametrize("rates", ["glauber", "metropolis"])
@pytest.mark.parametrize("J,H,T", [(1.0, 0.0, 4.5115), (1.0, 0.05, 4.4), (1.0, -0.05, 4.6), (0.0, 0.3, 1.0),
                                   (-0.5, 0.1, 2.0), (1.0, 0.0, 1e3)])
def test_rate_table_bitwise_equals_oracle(spkmc, rates, J, H, T):
    p = spkmc.make_params(16, 8, J=J, H=H, T=T, rates=rates)
    lib_tab = spkmc.rate_table(p)
    orc_tab = oracle.rate_table(J, H, T, 0 if rates == "glauber" else 1)
    assert np.array_equal(lib_tab.view(np.uint64), orc_tab.view(np.uint64))


def test_state_bytes_scale(spkmc):
    # packed 1024^3 with d = 32: bits of the spins, their halo copies, the slab
    # engine's counts (896 bytes per domain) and per-domain scratch
    p = spkmc.make_params(1024, 32, layout="packed")
    nb = spkmc.state_bytes(p)
    K = 32 ** 3
    assert nb >= 1024 ** 3 // 8 + K * 8 * 6 * 16 * 16 // 8 + K * 896
    assert nb < 1024 ** 3 // 8 * 1.8


def _c_layout(spkmc, tmp_path):
    """sizeof and offsetof of every field of the header's structs, from gcc."""
    structs = {"spkmc_params": spkmc.Params, "spkmc_record": spkmc.Record, "spkmc_obs": spkmc.Obs,
               "spkmc_info": spkmc.Info, "spkmc_batch_info": spkmc.BatchInfo,
               "spkmc_server_config": spkmc.ServerConfig, "spkmc_request_status": spkmc.RequestStatus,
               "spkmc_server_stats": spkmc.ServerStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "spkmc.h"', "int main(void) {"]
    for cname, ct in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in ct._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for ln in out.splitlines():
        a, b, c = ln.split()
        got[(a, b)] = int(c)
    return structs, got


def test_ctypes_mirrors_match_c_layout(spkmc, tmp_path):
    # the header compiles as C99 and every ctypes mirror has the same layout
    structs, got = _c_layout(spkmc, tmp_path)
    for cname, ct in structs.items():
        assert got[(cname, "size")] == C.sizeof(ct), cname
        for f, _ in ct._fields_:
            assert got[(cname, f)] == getattr(ct, f).offset, (cname, f)


def _server_cfg(spkmc, **kw):
    c = spkmc.ServerConfig()
    c.struct_size = C.sizeof(spkmc.ServerConfig)
    c.macro_cycles, c.max_live, c.inflight, c.wg_domains, c.reserved = 100, 16, 2, 0, 0
    for k, v in kw.items():
        setattr(c, k, v)
    return c


@pytest.mark.parametrize("kw", [dict(struct_size=20), dict(macro_cycles=0), dict(max_live=0), dict(max_live=5000),
                                dict(inflight=0), dict(inflight=9), dict(wg_domains=-1), dict(reserved=3)])
def test_server_config_validated(spkmc, kw):
    cfg = _server_cfg(spkmc, **kw)
    assert spkmc.lib.spkmc_server_reserved_bytes(C.byref(cfg)) == 0
    h = C.c_void_p()
    assert spkmc.lib.spkmc_server_create(C.byref(cfg), C.c_void_p(1 << 20), 1 << 30, None, C.byref(h)) == spkmc.E_INVAL
    assert not h.value
    assert spkmc.lib.spkmc_server_last_error(None)


def test_server_pool_checked_before_any_device_call(spkmc):
    cfg = _server_cfg(spkmc)
    res = spkmc.lib.spkmc_server_reserved_bytes(C.byref(cfg))
    assert res > 0 and res % 256 == 0
    assert res >= spkmc.lib.spkmc_batch_workspace_bytes(16)
    h = C.c_void_p()
    assert spkmc.lib.spkmc_server_create(C.byref(cfg), None, 1 << 30, None, C.byref(h)) == spkmc.E_INVAL
    assert spkmc.lib.spkmc_server_create(C.byref(cfg), C.c_void_p((1 << 20) + 8), 1 << 30, None,
                                         C.byref(h)) == spkmc.E_INVAL
    assert spkmc.lib.spkmc_server_create(C.byref(cfg), C.c_void_p(1 << 20), res - 1, None,
                                         C.byref(h)) == spkmc.E_RANGE
    assert not h.value


def test_server_calls_reject_null(spkmc):
    p = spkmc.make_params(32, 16)
    rid = C.c_uint64()
    assert spkmc.lib.spkmc_server_submit(None, C.byref(p), 10, 0, 0, -1.0, C.byref(rid)) == spkmc.E_INVAL
    assert spkmc.lib.spkmc_server_step(None, 0, None) == spkmc.E_INVAL
    assert spkmc.lib.spkmc_server_poll(None, 1, None) == spkmc.E_INVAL
    assert spkmc.lib.spkmc_server_release(None, 1) == spkmc.E_INVAL
    assert spkmc.lib.spkmc_server_clock(None) == 0.0
    spkmc.lib.spkmc_server_destroy(None)


def test_two_colours_sizes_four_lines_per_domain(spkmc):
    one = spkmc.state_bytes(spkmc.make_params(64, 16))
    two = spkmc.state_bytes(spkmc.make_params(64, 16, variant="two_colours"))
    K = (64 // 16) ** 3
    assert two - one >= 3 * K * (8 + 64) - 512  # R_k and histogram of three more lines per domain


def test_batch_calls_reject_bad_arguments(spkmc):
    """Batch and batch-graph calls check their arguments before any device call."""
    g = C.c_void_p()
    cyc = (C.c_uint64 * 1)(10)
    ws = C.c_void_p(0)
    assert spkmc.lib.spkmc_run_batch(None, 0, cyc, 0, 0, ws, 0, None) == spkmc.E_INVAL
    assert spkmc.lib.spkmc_batch_graph_create(None, 0, cyc, 0, 0, ws, 0, None, C.byref(g)) == spkmc.E_INVAL
    assert not g.value
    ctxs = (C.c_void_p * 1)(None)
    assert spkmc.lib.spkmc_batch_graph_create(ctxs, 1, cyc, 0, 0, ws, 0, None, None) == spkmc.E_INVAL
    assert spkmc.lib.spkmc_batch_graph_launch(None, 1) == spkmc.E_INVAL
    spkmc.lib.spkmc_batch_graph_destroy(None)
