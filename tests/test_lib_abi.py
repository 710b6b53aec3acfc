"""CPU checks of the C ABI: the library loads, exports every entry point that
include/lbell.h declares, and its host-only calls (defaults, arena sizing,
status strings, argument validation) behave as documented.  No GPU work."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbell.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbs?_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2403_05443_amd import lbell
    return lbell.load()


def test_every_declared_symbol_is_exported(lib):
    from paper_2403_05443_amd import lbell
    names = declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
        assert n in lbell.SIGNATURES, n


def test_config_default(lib):
    from paper_2403_05443_amd.lbell import Config
    cfg = Config()
    assert lib.lb_config_default(C.byref(cfg)) == 0
    assert cfg.lattice == 19 and cfg.collision == 0 and cfg.tau == 1.0
    assert cfg.rotation == 0
    assert abs(cfg.magic - 3 / 16) < 1e-15 and cfg.rho0 == 1.0 and cfg.storage == 1


def _cfg(lib, **kw):
    from paper_2403_05443_amd.lbell import Config
    cfg = Config()
    lib.lb_config_default(C.byref(cfg))
    for k, v in kw.items():
        setattr(cfg, k, v)
    return cfg


def test_arena_bytes(lib):
    from paper_2403_05443_amd.lbell import Box, make_box
    b = (Box * 1)(make_box(128, 128, 128))
    n32 = lib.lb_arena_bytes(C.byref(_cfg(lib)), 1, b)
    n16 = lib.lb_arena_bytes(C.byref(_cfg(lib, storage=2)), 1, b)
    n64 = lib.lb_arena_bytes(C.byref(_cfg(lib, storage=0)), 1, b)
    pops = 2 * 19 * 128 ** 3
    assert 4 * pops < n32 < 4 * pops * 1.2
    assert 2 * pops < n16 < n32 < n64
    two = (Box * 2)(make_box(32, 32, 32), make_box(40, 36, 44))
    assert lib.lb_arena_bytes(C.byref(_cfg(lib)), 2, two) > 2 * 19 * 4 * (32 ** 3 + 40 * 36 * 44)


@pytest.mark.parametrize("field,value", [("tau", 0.5), ("lattice", 15), ("collision", 5), ("storage", 9),
                                         ("rho0", 1.1), ("max_semi_axis", 200.0), ("rotation", 3),
                                         ("rotation", -1)])
def test_invalid_config_sizes_to_zero(lib, field, value):
    from paper_2403_05443_amd.lbell import Box, make_box
    b = (Box * 1)(make_box(32, 32, 32))
    assert lib.lb_arena_bytes(C.byref(_cfg(lib, **{field: value})), 1, b) == 0


def test_invalid_boxes(lib):
    from paper_2403_05443_amd.lbell import Box, make_box
    assert lib.lb_arena_bytes(C.byref(_cfg(lib)), 1, (Box * 1)(make_box(3, 32, 32))) == 0
    assert lib.lb_arena_bytes(C.byref(_cfg(lib)), 1,
                              (Box * 1)(make_box(8, 8, 8, walls=True, wall_lo=(0, 0.1, 0)))) == 0
    assert lib.lb_arena_bytes(C.byref(_cfg(lib)), 1, (Box * 1)(make_box(8, 8, 8, init="couette"))) == 0
    assert lib.lb_arena_bytes(C.byref(_cfg(lib)), 0, (Box * 1)(make_box(8, 8, 8))) == 0


def test_status_strings_and_null_handling(lib):
    assert lib.lb_status_str(0) == b"ok"
    assert lib.lb_status_str(-5) == b"particle overlap"
    assert lib.lb_status_str(-99) == b"unknown status"
    assert lib.lb_step(None, 1) == -1
    assert lib.lb_destroy(None) == -1
    assert lib.lb_last_error(None) == b""
    from paper_2403_05443_amd.lbell import Box, make_box
    out = C.c_void_p()
    # a misaligned / null arena is rejected before any device call
    assert lib.lb_init(C.byref(_cfg(lib)), 1, (Box * 1)(make_box(8, 8, 8)), None, 0, None,
                       C.byref(out)) == -1
