"""The C ABI on the host: the library loads, exports every function the
header declares, and validates grids and options before any device work."""
import math

import pytest

from paper_0904_4887_amd import binding as B
from paper_0904_4887_amd import workloads as W


def test_library_exports_every_header_symbol():
    lib = B.lib()
    names = B.header_symbols()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name


def test_default_opts():
    o = B.default_opts()
    assert o.precision == 0 and o.pre == 2 and o.post == 2 and o.cycles == 1
    assert math.isnan(o.z_wet_lo) and math.isnan(o.z_wet_hi)
    assert o.tol == 1e-10 and o.restart == 10 and o.warm_start == 0 and o.profile == 0
    assert o.smoother == 1 and o.fft_fp32 == 0 and o.order == 2 and o.smooth6 == 0 and o.krylov_fp32 == 0
    assert o.krylov_fp16 == 0 and o.semi_ratio == math.sqrt(2.0)


@pytest.mark.parametrize("n", [(30, 32, 64), (32, 32, 6), (32, 32, 70), (32, 32, 8192), (33, 32, 64)])
def test_plan_rejects_bad_grid_sizes(n):
    with pytest.raises(B.DWPError) as e:
        B.plan(n, (10.0, 10.0, 20.0))
    assert e.value.status == B.DWP_EINVAL


@pytest.mark.parametrize("kw", [dict(precision=2), dict(tol=0.0), dict(tol=1.5), dict(restart=0),
                                dict(restart=64), dict(cycles=-1), dict(cycles=65), dict(pre=0, post=0), dict(max_outer=0),
                                dict(z_wet_lo=8.0, z_wet_hi=8.5), dict(z_wet_lo=0.0, z_wet_hi=20.0),
                                dict(profile=3), dict(scaled_dry=3), dict(fft_fp32=2),
                                dict(fft_fp32=1, precision=0), dict(smoother=3), dict(order=4),
                                dict(smooth6=2), dict(smooth6=1), dict(smooth6=1, order=2),
                                dict(krylov_fp32=2), dict(krylov_fp32=1, precision=0),
                                dict(krylov_fp32=1, precision=1, order=6),
                                dict(krylov_fp32=1, precision=1, restart=17),
                                dict(krylov_fp16=2), dict(krylov_fp16=1, precision=1),
                                dict(krylov_fp16=1, krylov_fp32=1, precision=1, order=6, cycles=0),
                                dict(semi_ratio=0.5), dict(semi_ratio=65.0), dict(semi_ratio=float("nan"))])
def test_plan_rejects_bad_options(kw):
    with pytest.raises(B.DWPError) as e:
        B.plan((32, 32, 64), (10.0, 10.0, 20.0), **kw)
    assert e.value.status == B.DWP_EINVAL


def test_plan_rejects_bad_lengths():
    for L in [(0.0, 10.0, 20.0), (10.0, -1.0, 20.0), (10.0, 10.0, float("nan"))]:
        with pytest.raises(B.DWPError):
            B.plan((32, 32, 64), L)


def test_plan_wet_slab_and_hierarchy():
    # tanh box, dry z < 8 A: planes 26..63, moved down one plane so that 40
    # intervals halve three times
    p = B.plan((32, 32, 64), (10.0, 10.0, 20.0), z_wet_lo=8.0, z_wet_hi=20.0)
    assert (p["k_w0"], p["k_w1"]) == (25, 64)
    assert p["levels"] == [(32, 32, 39), (16, 16, 19), (8, 8, 9)]
    # slab: hz / hx = 1.69 > sqrt 2, so the first coarsening is in x, y only
    w = W.slab((96, 96, 192))
    p = B.plan(w.n, w.L, z_wet_lo=w.z_wet[0], z_wet_hi=w.z_wet[1])
    assert p["k_w1"] == 192 and p["k_w0"] <= 68
    assert p["levels"][0] == (96, 96, 192 - p["k_w0"]) and p["levels"][1][2] == p["levels"][0][2]
    assert all(l[0] % 2 == 0 and l[1] % 2 == 0 for l in p["levels"])
    last = p["levels"][-1]
    assert last[0] * last[1] * last[2] <= 1024
    # semi_ratio 2 > 1.69: every coarsening halves z too (the levels' z
    # interval counts halve: nw + 1 -> (nw + 1) / 2)
    q = B.plan(w.n, w.L, z_wet_lo=w.z_wet[0], z_wet_hi=w.z_wet[1], semi_ratio=2.0)
    assert q["levels"][0] == p["levels"][0]
    assert all(c[2] + 1 == (f[2] + 1) // 2 for f, c in zip(q["levels"], q["levels"][1:]))
    assert q["levels"][1][2] < p["levels"][1][2]
    # a wet slab that wraps through z = 0
    p = B.plan((32, 32, 64), (10.0, 10.0, 20.0), z_wet_lo=8.0, z_wet_hi=20.0 + 2 * 20.0 / 64)
    assert p["k_w1"] == 66 and p["k_w1"] - p["k_w0"] == p["levels"][0][2]


def test_create_without_device_fails_cleanly():
    import ctypes as C
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible")
    except Exception:
        pass
    h = C.c_void_p()
    st = B.lib().dwp_create(C.byref(h), 0, None)
    assert st != B.DWP_OK and not h.value
    assert len(B.lib().dwp_last_error(None)) > 0
    # NULL contexts are rejected, never dereferenced
    assert B.lib().dwp_solve(None, None, None, None, None) == B.DWP_EINVAL


def test_plan_accepts_float32_krylov_vectors_where_supported():
    # second order at any cycle count; sixth order with the FFT dry update alone
    for kw in (dict(krylov_fp32=1, precision=1), dict(krylov_fp32=1, precision=1, restart=16),
               dict(krylov_fp32=1, precision=1, order=6, cycles=0),
               dict(krylov_fp32=1, krylov_fp16=1, precision=1)):
        B.plan((32, 32, 64), (10.0, 10.0, 20.0), **kw)
