"""CPU checks of the C ABI: the library loads, exports every declared symbol, validates arguments on
the host before touching the device, and its host-side bank agrees with the oracle's."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2601_09417_amd import _lib as L
from paper_2601_09417_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "vbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vbm_[a-z0-9_]+)\s*\(", src)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = L.load()
    declared = _declared_functions()
    assert len(declared) >= 16
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(L.EXPORTS)
    assert b"gfx950" in lib.vbm_version()


def test_null_and_size_checks_return_before_launch():
    lib = L.load()
    assert lib.vbm_dwt3d(None, 32, 1, 0, None, None, None, 0, None) == -1
    # G not divisible by 2^J
    assert lib.vbm_dwt3d(1, 36, 3, 0, None, 1, 1, 1 << 30, None) == -1
    # unknown wavelet
    assert lib.vbm_dwt3d(1, 32, 1, 7, None, 1, 1, 1 << 30, None) == -2
    # workspace too small
    assert lib.vbm_dwt3d(1, 32, 1, 0, None, 1, 1, 16, None) == -3
    g = L.vbm_gaussians(1, 1, 1, 1, 1, 10)
    opts = L.vbm_build_opts(0, 0.5, 1e-3, 0.99)
    assert lib.vbm_build_gaussians(1, 16, 2, 1, 16 ** 3 + 1, C.byref(opts), g, None, 1, 1 << 30, None) == -1
    assert lib.vbm_build_gaussians(1, 16, 2, 1, 20, C.byref(opts), g, None, 1, 1 << 30, None) == -1  # stride < K
    assert b"stride" in lib.vbm_last_error()
    assert lib.vbm_adam_step(10, 5, 1, 1, 1, g, g, None, None, None) == -1


def _cam(w=64, h=48):
    import vbm_inputs as vi
    return vi.orbit_cameras(1, w, h)[0]


def test_plan_validation_and_layout():
    lib = L.load()
    views = (L.vbm_view * 1)(api.make_view(_cam()))
    so = np.array([0, 100], np.int64)
    p = L.vbm_plan()
    for tile, bits, cap, mode, expect in [(12, 8, 100, 0, -2), (16, 3, 100, 0, -1), (16, 8, 0, 0, -1),
                                          (16, 8, 100, 9, -1), (16, 8, 100, 0, 0), (32, 4, 7, 1, 0)]:
        sch = L.vbm_schedule(tile, bits, cap, mode, 0)
        st = lib.vbm_plan_make(views, 1, so.ctypes.data_as(C.POINTER(C.c_int64)), 1, C.byref(sch), C.byref(p), None)
        assert st == expect, (tile, bits, cap, mode, st)
    assert p.n_items == 100 and p.n_tiles == 2 * 2 and p.n_pixels == 64 * 48 and p.tile_key_bits == 2
    n_regions = 22                                        # 20 documented, then mask and tile-order scratch
    offs = [p.region_offset[r] for r in range(n_regions)]
    sizes = [p.region_bytes[r] for r in range(n_regions)]
    for r in range(n_regions - 1):
        assert offs[r] + sizes[r] <= offs[r + 1]
        assert offs[r] % 256 == 0
    assert p.ws_bytes >= offs[-1] + sizes[-1]
    assert sizes[19] == 32 * p.n_items
    assert sizes[21] == 16 * p.n_tiles
    bad = (L.vbm_view * 1)(api.make_view(_cam()))
    bad[0].scene = 3
    sch = L.vbm_schedule(16, 8, 100, 0, 0)
    assert lib.vbm_plan_make(bad, 1, so.ctypes.data_as(C.POINTER(C.c_int64)), 1, C.byref(sch), C.byref(p), None) == -1
    bad[0].scene = 0
    bad[0].fx = -1.0
    assert lib.vbm_plan_make(bad, 1, so.ctypes.data_as(C.POINTER(C.c_int64)), 1, C.byref(sch), C.byref(p), None) == -1


def test_render_rejects_small_workspace():
    lib = L.load()
    views = (L.vbm_view * 1)(api.make_view(_cam()))
    so = np.array([0, 100], np.int64)
    p = L.vbm_plan()
    sch = L.vbm_schedule(16, 8, 1000, 0, 0)
    assert lib.vbm_plan_make(views, 1, so.ctypes.data_as(C.POINTER(C.c_int64)), 1, C.byref(sch), C.byref(p), None) == 0
    g = L.vbm_gaussians(1, 1, 1, 1, 1, 100)
    assert lib.vbm_render_fwd(C.byref(p), 1, g, 1, 1, 1, 1, 1, p.ws_bytes - 1, None) == -3
    g.stride = 50
    assert lib.vbm_render_fwd(C.byref(p), 1, g, 1, 1, 1, 1, 1, p.ws_bytes, None) == -1


@pytest.mark.parametrize("wav,J", [("haar", 4), ("bior4.4", 3)])
def test_host_bank_matches_oracle_bank(wav, J):
    from oracle import bank as obank
    ref = obank.build_bank(wav, J)
    entries, packed = api.bank_build(wav, J)
    assert len(entries) == len(ref) == 7 * J + 1
    for e, r in zip(entries, ref):
        assert (e["j"], e["o"]) == (r.j, r.o)
        assert e["roi_size"] == r.roi_size
        assert abs(e["w"] - r.w) <= 1e-12 * r.w
        assert np.allclose(e["u"], r.u, atol=1e-10)
        S = np.array([[e["sigma"][0], e["sigma"][3], e["sigma"][4]], [e["sigma"][3], e["sigma"][1], e["sigma"][5]],
                      [e["sigma"][4], e["sigma"][5], e["sigma"][2]]])
        assert np.allclose(S, r.sigma, rtol=1e-12, atol=1e-12)
        assert np.allclose(e["scale"], r.scale, rtol=1e-12)
    for i, e in enumerate(entries):
        expect = np.concatenate([[e["w"]], e["u"], e["scale"], e["quat"], [0.0]]).astype(np.float32)
        assert np.array_equal(packed[i], expect)
