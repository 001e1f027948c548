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
    inst = pga.InstanceC(8, 4, 0x1000, None, None, 0x1000, 0x1000, 0x1000, None,
                         pga.Params(4, 2, 0, 0, 0, 0, 0))           # E >= P
    arr = (pga.InstanceC * 1)(inst)
    assert lib.pga_evolve(None, arr, 1, 1, 0, 0, wsp, 1 << 16, None, None) == -1
    assert lib.pga_evolve_ws_bytes(arr, 1, 0) == 0
    arr[0].prm.elites = 1
    arr[0].prm.tournament = 3
    assert lib.pga_evolve_ws_bytes(arr, 1, 0) == 0
    arr[0].prm.tournament = 2
    assert lib.pga_evolve_ws_bytes(arr, 1, 0) > 8 * 4 * 8
    assert lib.pga_evolve_ws_bytes(arr, 1, 1) == 0      # MFMA form needs hi/lo
    # best: P < 1
    assert lib.pga_best(fake, fake, 0, 4, None, None, None, wsp, 1 << 16, None) == -1


def test_workspace_sizes(lib):
    assert lib.pga_split_ld(1) == 32 and lib.pga_split_ld(32) == 32 and lib.pga_split_ld(33) == 64
    assert lib.pga_fitness_ws_bytes(1024, 4096, 0) >= 1024 * 4096 * 8
    assert lib.pga_correlate_ws_bytes(100) >= 1600
    assert lib.pga_best_ws_bytes(18) >= 19 * 4
    assert lib.pga_strerror(-2).decode().startswith("workspace")
