"""CPU-only checks of the C ABI: the library loads, exports every symbol that
include/pga.h declares, and rejects bad arguments on the host before touching
the GPU. No compute call is made here."""
import ctypes as ct
import os
import re

import pytest

from paper_1403_4099_amd import pga

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pga.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pga.LIB_PATH):
        from paper_1403_4099_amd import build
        build.build()
    return pga.load()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pga_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("pga_correlate", "pga_fitness", "pga_evolve", "pga_best", "pga_split"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(_declared()) == sorted(pga.SYMBOLS)


def test_host_side_argument_errors(lib):
    vp = ct.c_void_p
    ws = ct.create_string_buffer(1 << 16)
    wsp = ct.cast(ws, vp)
    fake = vp(0x1000)   # never dereferenced: every call below fails its argument check first
    # fitness: N < 1, bad form, missing hi/lo for the MFMA form, N > N_MAX, small workspace
    assert lib.pga_fitness(fake, None, None, 0, fake, 4, 0, fake, None, None, None, wsp, 1 << 16, None) == -1
    assert lib.pga_fitness(fake, None, None, 8, fake, 4, 7, fake, None, None, None, wsp, 1 << 16, None) == -1
    assert lib.pga_fitness(fake, None, None, 8, fake, 4, 1, fake, None, None, None, wsp, 1 << 16, None) == -1
    assert lib.pga_fitness(fake, None, None, pga.N_MAX + 1, fake, 4, 0, fake, None, None, None, wsp,
                           1 << 16, None) == -4
    assert lib.pga_fitness(fake, None, None, 64, fake, 64, 0, fake, None, None, None, wsp, 16, None) == -2
    # P = 0 is a no-op that succeeds without touching anything
    assert lib.pga_fitness(None, None, None, 8, None, 0, 0, None, None, None, None, None, 0, None) == 0
    # correlate: T < 2, ld < T, hi without lo, missing workspace
    assert lib.pga_correlate(fake, 4, 1, 1, fake, None, None, None, wsp, 1 << 16, None) == -1
    assert lib.pga_correlate(fake, 4, 8, 4, fake, None, None, None, wsp, 1 << 16, None) == -1
    assert lib.pga_correlate(fake, 4, 8, 8, fake, fake, None, None, wsp, 1 << 16, None) == -1
    assert lib.pga_correlate(fake, 4, 8, 8, fake, None, None, None, None, 0, None) == -2
    # evolve: null ctx; bad instance parameters
    inst = pga.InstanceC(8, 4, 0x1000, None, None, 0x1000, 0x1000, 0x1000, None, None,
                         pga.Params(4, 2, 0, 0, 0, 0, 0, 0, 0, 1e-5))   # E >= P
    arr = (pga.InstanceC * 1)(inst)
    assert lib.pga_evolve(None, arr, 1, 1, 0, 0, wsp, 1 << 16, None, None) == -1
    assert lib.pga_evolve_ws_bytes(arr, 1, 0) == 0
    arr[0].prm.elites = 1
    arr[0].prm.tournament = 3
    assert lib.pga_evolve_ws_bytes(arr, 1, 0) == 0
    arr[0].prm.tournament = 2
    assert lib.pga_evolve_ws_bytes(arr, 1, 0) > 8 * 4 * 8
    assert lib.pga_evolve_ws_bytes(arr, 1, 1) == 0      # MFMA form needs hi/lo
    # termination test: needs a state buffer, a non-negative stall count, a known selection, a tolerance
    arr[0].prm.stall_gens = 50
    assert lib.pga_evolve_ws_bytes(arr, 1, 0) == 0
    arr[0].term = 0x2000
    assert lib.pga_evolve_ws_bytes(arr, 1, 0) > 0
    arr[0].prm.stall_gens = -1
    assert lib.pga_evolve_ws_bytes(arr, 1, 0) == 0
    arr[0].prm.stall_gens = 50
    arr[0].prm.selection = 2
    assert lib.pga_evolve_ws_bytes(arr, 1, 0) == 0
    arr[0].prm.selection = 1                            # SUS: tournament size is not used
    arr[0].prm.tournament = 5
    sus_bytes = lib.pga_evolve_ws_bytes(arr, 1, 0)
    arr[0].prm.selection = 0
    arr[0].prm.tournament = 2
    assert sus_bytes >= lib.pga_evolve_ws_bytes(arr, 1, 0) + 4 * (4 + 8)
    arr[0].prm.tol = float("nan")
    assert lib.pga_evolve_ws_bytes(arr, 1, 0) == 0
    # allocation-free fitness: same argument checks; a workspace need above the static scratch is refused
    assert lib.pga_fitness_noalloc(fake, None, None, 0, fake, 4, 0, fake, None, None, None, None) == -1
    assert lib.pga_fitness_noalloc(fake, None, None, 8, fake, 4, 7, fake, None, None, None, None) == -1
    assert lib.pga_fitness_noalloc(fake, None, None, pga.N_MAX + 1, fake, 4, 0, fake, None, None, None,
                                   None) == -4
    assert lib.pga_fitness_noalloc(None, None, None, 8, None, 0, 0, None, None, None, None, None) == 0
    assert lib.pga_fitness_ws_bytes(2048, 4096, 0) > lib.pga_fitness_noalloc_max_bytes()
    assert lib.pga_fitness_noalloc(fake, None, None, 2048, fake, 4096, 0, fake, None, None, None, None) == -4
    assert lib.pga_fitness_ws_bytes(1024, 4096, 1) <= lib.pga_fitness_noalloc_max_bytes() == 40 << 20
    # graph count of a null context
    assert lib.pga_ctx_graphs(None) == -1
    # best: P < 1
    assert lib.pga_best(fake, fake, 0, 4, None, None, None, wsp, 1 << 16, None) == -1


def test_variant_table_host_side(lib):
    # two forms, each with variant 0 as the default; the table is keyed by (form, N/64, log2 P)
    assert lib.pga_variant_count(0) >= 2 and lib.pga_variant_count(1) >= 2
    assert lib.pga_variant_count(7) == -1
    ipg, xcd = ct.c_int32(), ct.c_int32()
    # variant 0 (the default) deals tiles to the XCDs in contiguous ranges, column pairs fastest
    # MFMA kinds: 0 register one-hot (the default), 1 compacted columns, 2 one-hot from the LDS table
    kind = ct.c_int32()
    assert lib.pga_variant_info(1, 0, ct.byref(ipg), ct.byref(xcd), ct.byref(kind)) == 0 and xcd.value == 1 \
        and ipg.value == 8 and kind.value == 0
    kinds = set()
    for v in range(lib.pga_variant_count(1)):
        assert lib.pga_variant_info(1, v, None, None, ct.byref(kind)) == 0
        kinds.add(kind.value)
    assert kinds == {0, 1, 2}
    assert lib.pga_variant_info(0, 0, ct.byref(ipg), ct.byref(xcd), None) == 0 and xcd.value == 1 and ipg.value == 8
    assert lib.pga_variant_info(1, lib.pga_variant_count(1), None, None, None) == -1
    assert lib.pga_tune_get(1, 1024, 4096) == 0
    assert lib.pga_tune_set(1, 1024, 4096, 2) == 0
    assert lib.pga_tune_get(1, 1000, 3000) == 2           # same bucket
    assert lib.pga_tune_get(1, 1100, 4096) == 0           # another N bucket
    assert lib.pga_tune_get(0, 1024, 4096) == 0           # another form
    assert lib.pga_tune_set(1, 1024, 4096, -1) == 0
    assert lib.pga_tune_get(1, 1024, 4096) == 0
    assert lib.pga_tune_set(1, 1024, 4096, 99) == -1
    # a variant that cannot hold N falls back to the first variant that can
    big = [v for v in range(lib.pga_variant_count(1))
           if lib.pga_variant_info(1, v, ct.byref(ipg), ct.byref(xcd), None) == 0 and ipg.value == 16][0]
    first_fit = lib.pga_tune_get(1, 4096, 512)
    assert first_fit != big
    assert lib.pga_tune_set(1, 4096, 512, big) == 0 and lib.pga_tune_get(1, 4096, 512) == first_fit
    assert lib.pga_tune_set(1, 4096, 512, -1) == 0
    assert lib.pga_tune_get(1, 1024, 512) == 0
    # tune: argument and workspace errors come back before any GPU work
    assert lib.pga_tune(None, None, None, 64, None, 64, 0, 0, None, 0, None, None, None) == -1
    fake = ct.c_void_p(0x1000)
    assert lib.pga_tune(fake, None, None, 64, fake, 64, 0, 3, None, 0, None, None, None) == -2
    assert lib.pga_tune_ws_bytes(64, 64, 0) > lib.pga_fitness_ws_bytes(64, 64, 0)


def test_workspace_sizes(lib):
    assert lib.pga_split_ld(1) == 32 and lib.pga_split_ld(32) == 32 and lib.pga_split_ld(33) == 64
    assert lib.pga_fitness_ws_bytes(1024, 4096, 0) >= 1024 * 4096 * 8
    assert lib.pga_correlate_ws_bytes(100) >= 1600
    assert lib.pga_best_ws_bytes(18) >= 19 * 4
    assert lib.pga_strerror(-2).decode().startswith("workspace")


def test_peak_mfma_rejects_bad_arguments():
    """The measurement aid checks its arguments before touching the GPU."""
    L = pga.load()
    flops = ct.c_double()
    assert L.pga_peak_mfma_bf16(None, 1, 1, ct.byref(flops), None) == -1  # PGA_ERR_ARG
    buf = ct.create_string_buffer(64)
    assert L.pga_peak_mfma_bf16(ct.cast(buf, ct.c_void_p), 0, 1, None, None) == -1  # PGA_ERR_ARG
    assert L.pga_peak_mfma_bf16(ct.cast(buf, ct.c_void_p), 1, 0, None, None) == -1  # PGA_ERR_ARG
    # the pipe-mix loops: a null sink, an unknown mode or an empty launch
    assert L.pga_pipe_mix(None, 1, 1, 1, None) == -1
    for mode in (0, 6, 7, 8, 9, 12, 15, 16, -1):
        assert L.pga_pipe_mix(ct.cast(buf, ct.c_void_p), mode, 1, 1, None) == -1, mode
    assert L.pga_pipe_mix(ct.cast(buf, ct.c_void_p), 1, 0, 1, None) == -1
    assert L.pga_pipe_mix(ct.cast(buf, ct.c_void_p), 1, 1, 0, None) == -1


def test_route_limit_is_host_state_with_checked_range(lib):
    """The cluster-pair route limit is a host-side setting: set, read back, range-checked."""
    prev = pga.route_get()
    assert prev == 1.0 / 64.0                        # PGA_ROUTE_FRAC_DEFAULT
    try:
        for bad in (-0.1, 1.5, float("nan")):
            assert lib.pga_route_set(bad) == -1      # PGA_ERR_ARG
            assert pga.route_get() == prev
        for ok in (0.0, 0.25, 1.0):
            assert lib.pga_route_set(ok) == 0
            assert pga.route_get() == ok
        with pga.route(0.5):
            assert pga.route_get() == 0.5
        assert pga.route_get() == 1.0
    finally:
        pga.route_set(prev)


def test_tuning_table_persists_to_a_file(lib, tmp_path):
    """The tuning table round-trips through its text file; a malformed file is rejected whole."""
    f = tmp_path / "tune.txt"
    try:
        assert pga.tune_get("bf16x2", 300, 512) == 0
        pga.tune_set("bf16x2", 300, 512, 4)
        pga.tune_set("fp64", 1024, 4096, 1)
        n = pga.tune_save(str(f))
        assert n >= 2
        text = f.read_text()
        assert "1 5 9 4" in text and "0 16 12 1" in text          # form ceil(N/64) ceil(log2 P) variant
        pga.tune_set("bf16x2", 300, 512, -1)
        pga.tune_set("fp64", 1024, 4096, -1)
        assert pga.tune_get("bf16x2", 300, 512) == 0
        assert pga.tune_load(str(f)) == n
        assert pga.tune_get("bf16x2", 300, 512) == 4 and pga.tune_get("fp64", 1000, 3000) == 1
        bad = tmp_path / "bad.txt"
        bad.write_text("1 5 9 2\n1 5 9 99\n")                    # variant out of range
        pga.tune_set("bf16x2", 300, 512, -1)
        assert lib.pga_tune_load(str(bad).encode()) == -1
        assert pga.tune_get("bf16x2", 300, 512) == 0                # nothing of it applied
        assert lib.pga_tune_load(str(tmp_path / "missing.txt").encode()) == -1
    finally:
        pga.tune_set("bf16x2", 300, 512, -1)
        pga.tune_set("fp64", 1024, 4096, -1)
