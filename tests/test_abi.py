"""Host-side checks of the C ABI (no GPU needed): the built library exports
every entry point include/*.h declares, and parameter validation returns the
documented error codes before any device work."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(lbm_axi_\w+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    from paper_1310_1871_amd import lbm_axi as L
    lib = ctypes.CDLL(L.LIB_PATH)
    names = _declared()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_parameter_validation():
    from paper_1310_1871_amd import lbm_axi as L
    good = L.make_params(64, 32)
    assert L.workspace_bytes(good) > 2 * 9 * 64 * 32 * 8
    for field, value, msg in [("nz", 0, "nz"), ("nr", 5, "nr"), ("tau", 0.5, "tau"), ("wall", 2, "wall"),
                              ("axisym", 3, "axisym"), ("precision", 7, "precision"), ("psi_rho0", 0.0, "psi_rho0"),
                              ("flags", 1, "flags"), ("flags", 32, "flags"), ("flags", 3, "flags")]:
        p = L.make_params(64, 32)
        setattr(p, field, value)
        assert L.workspace_bytes(p) == 0
        assert msg in L.last_error()
    for flags in (L.FLAG_GUO, L.FLAG_NO_WALL_DERIV, L.FLAG_GUO | L.FLAG_NO_WALL_DERIV, L.FLAG_ZWALLS,
                  L.FLAG_ZWALLS | L.FLAG_GUO | L.FLAG_NO_WALL_DERIV):
        assert L.workspace_bytes(L.make_params(64, 32, flags=flags)) == L.workspace_bytes(good)
    assert L.workspace_bytes(L.make_params(7, 32, flags=L.FLAG_ZWALLS)) == 0 and "nz" in L.last_error()
    # the mid-link source needs 3 nz nr doubles more, and no closed z ends
    extra = L.workspace_bytes(L.make_params(64, 32, flags=L.FLAG_MIDLINK)) - L.workspace_bytes(good)
    assert 3 * 64 * 32 * 8 <= extra < 3 * 64 * 32 * 8 + 512
    assert L.workspace_bytes(L.make_params(64, 32, flags=L.FLAG_MIDLINK | L.FLAG_ZWALLS)) == 0
    assert "MIDLINK" in L.last_error()


def test_stability_rule_warning():
    """Sec. II.D: a density ratio of about 35 (G >= -6) is the scheme's
    stability limit as a rule of thumb.  check_params (no device) returns the
    positive warning code LBM_AXI_WARN_STABILITY for G < -6, with a message,
    and OK at G = -6; invalid parameters still return their error."""
    import warnings
    from paper_1310_1871_amd import lbm_axi as L
    assert L.lib.lbm_axi_check_params(ctypes.byref(L.make_params(64, 32, G=-6.0))) == L.OK
    assert L.lib.lbm_axi_check_params(ctypes.byref(L.make_params(64, 32, G=-5.5))) == L.OK
    assert L.lib.lbm_axi_check_params(ctypes.byref(L.make_params(64, 32, G=-6.5))) == L.WARN_STABILITY
    assert "-6.5" in L.last_error() and "stability" in L.last_error()
    assert L.lib.lbm_axi_check_params(ctypes.byref(L.make_params(64, 32, G=-6.5, tau=0.4))) == L.EINVAL
    assert L.lib.lbm_axi_check_params(None) == L.EINVAL
    # the workspace size is unaffected, and the binding turns the code into a warning
    assert L.workspace_bytes(L.make_params(64, 32, G=-6.5)) == L.workspace_bytes(L.make_params(64, 32))
    with warnings.catch_warnings(record=True) as w:
        warnings.simplefilter("always")
        assert L.check_params(L.make_params(64, 32, G=-7.0)) == L.WARN_STABILITY
    assert any(issubclass(x.category, L.StabilityWarning) for x in w)
    with pytest.raises(L.LbmAxiError):
        L.check_params(L.make_params(64, 5))


def test_fp32_workspace_is_half():
    from paper_1310_1871_amd import lbm_axi as L
    a = L.workspace_bytes(L.make_params(4096, 512, precision=L.FP64))
    b = L.workspace_bytes(L.make_params(4096, 512, precision=L.FP32_SHIFTED, rho_ref=1.0))
    assert abs(a / b - 2.0) < 0.01


def test_create_rejects_bad_pointers_without_device_work():
    from paper_1310_1871_amd import lbm_axi as L
    p = L.make_params(64, 32)
    h = ctypes.c_void_p()
    rc = L.lib.lbm_axi_create(ctypes.byref(p), None, None, None, None, 0, None, ctypes.byref(h))
    assert rc == L.EINVAL and "rho0" in L.last_error()
    rc = L.lib.lbm_axi_create(ctypes.byref(p), ctypes.c_void_p(4096), None, None, ctypes.c_void_p(4096), 16,
                              None, ctypes.byref(h))
    assert rc == L.ENOMEM and "workspace too small" in L.last_error()
    rc = L.lib.lbm_axi_create(ctypes.byref(p), ctypes.c_void_p(4096), None, None, ctypes.c_void_p(4100),
                              1 << 30, None, ctypes.byref(h))
    assert rc == L.EINVAL and "aligned" in L.last_error()
    assert L.lib.lbm_axi_step(None, 1) == L.EINVAL
    n = ctypes.c_int32()
    assert L.lib.lbm_axi_drops(None, 1.0, 4, ctypes.byref(n), None, None) == L.EINVAL
    assert L.lib.lbm_axi_set_open(None, 9, 1.0, None, None, 20, 1.0) == L.EINVAL
    assert L.lib.lbm_axi_populations(None, ctypes.c_void_p(4096)) == L.EINVAL
    assert L.lib.lbm_axi_set_kernel(None, L.KERNEL_STRIP, 48) == L.EINVAL
    L.lib.lbm_axi_destroy(None)


def test_ray_weights_host_builder_matches_oracle():
    """The library's host-side construction of the ray-integral interface
    radius (a reading of the shape observable) equals the oracle's own
    construction of the same definition."""
    import numpy as np
    import oracle.diagnostics as D
    from paper_1310_1871_amd import lbm_axi as L
    lib = L.lib
    i32, dbl = ctypes.c_int32, ctypes.c_double
    for nz, nr, zc in [(64, 32, 32.0), (256, 128, 128.0), (37, 11, 12.3)]:
        th = [(k + 0.5) * np.pi / 16 for k in range(16)]
        s_max = min(nz / 2.0, float(nr)) - 1.0
        tha = (dbl * 16)(*th)
        nnz, nn = i32(), i32()
        assert lib.lbm_axi_ray_weights(nz, nr, dbl(zc), tha, 16, dbl(0.5), dbl(s_max), 0, None, None, None, None,
                                       None, None, None, ctypes.byref(nnz), ctypes.byref(nn)) == 0
        cap = nnz.value
        rp, col, val = (i32 * 17)(), (i32 * cap)(), (dbl * cap)()
        npt, nodes, nrow, nval = (i32 * (nn.value + 1))(), (i32 * nn.value)(), (i32 * cap)(), (dbl * cap)()
        assert lib.lbm_axi_ray_weights(nz, nr, dbl(zc), tha, 16, dbl(0.5), dbl(s_max), cap, rp, col, val, npt, nodes,
                                       nrow, nval, ctypes.byref(nnz), ctypes.byref(nn)) == 0
        ref = D.interface_radius_weights(nz, nr, zc, th, ds=0.5, s_max=s_max)
        for m, (idx, w) in enumerate(ref):
            lo, hi = rp[m], rp[m + 1]
            assert list(col[lo:hi]) == list(idx)
            assert np.allclose(np.array(val[lo:hi]), w, rtol=1e-14, atol=1e-15)
        # node-major copy holds the same entries
        tot = sum(val[k] for k in range(cap))
        assert abs(tot - sum(nval[k] for k in range(cap))) < 1e-9
        small = (i32 * 1)()
        assert lib.lbm_axi_ray_weights(nz, nr, dbl(zc), tha, 16, dbl(0.5), dbl(s_max), 1, rp, small, val, npt,
                                       nodes, nrow, nval, ctypes.byref(nnz), ctypes.byref(nn)) == L.ENOMEM


def test_ray_weights_rejects_bad_geometry():
    """The host-side ray builder refuses, with LBM_AXI_EINVAL and a message,
    every input that would reach an undefined float-to-int conversion or a
    runaway sample count: non-finite zc, ds, s_max or angle, ds <= 0,
    s_max < 0, |zc| + s_max > 1e9, more than 2^24 samples per ray, a grid
    beyond 32-bit node indices.  Valid geometry still builds."""
    import math
    from paper_1310_1871_amd import lbm_axi as L
    lib = L.lib
    i32, dbl = ctypes.c_int32, ctypes.c_double
    nnz, nn = i32(), i32()

    def call(nz=64, nr=32, zc=32.0, th=(0.3, 1.2), ds=0.5, s_max=20.0):
        tha = (dbl * len(th))(*th)
        return lib.lbm_axi_ray_weights(nz, nr, dbl(zc), tha, len(th), dbl(ds), dbl(s_max), 0, None, None, None,
                                       None, None, None, None, ctypes.byref(nnz), ctypes.byref(nn))

    assert call() == L.OK and nnz.value > 0
    bad = [dict(zc=math.nan), dict(zc=math.inf), dict(ds=math.nan), dict(ds=0.0), dict(ds=-0.5),
           dict(s_max=math.inf), dict(s_max=math.nan), dict(s_max=-1.0), dict(th=(0.3, math.nan)),
           dict(zc=2e9), dict(s_max=1e7, ds=0.5), dict(nz=1 << 20, nr=1 << 12)]
    for kw in bad:
        assert call(**kw) == L.EINVAL, kw
        assert "ray weights" in L.last_error(), kw
    # the limits themselves are accepted
    assert call(s_max=float(1 << 23), ds=0.5, th=(0.3,), nz=64, nr=32) == L.OK


def test_adjoint_helpers_reject_bad_arguments_without_device_work():
    """The adjoint's helper calls check their arguments before any launch
    and say why in last_error: NULL pointers, negative counts, empty grids,
    a grid beyond 32-bit indices for the ray VJP (whose kernel adds into
    the nine nz nr planes of lam), and equal or non-finite phase
    densities."""
    import math
    from paper_1310_1871_amd import adjoint as A
    from paper_1310_1871_amd import lbm_axi as L
    lib = A._lib
    p = ctypes.c_void_p(4096)  # never dereferenced: every call below fails its checks first
    cases = [
        (lambda: lib.lbm_axi_init_vjp(None, None, None, 8, 8, p, None), "init_vjp"),
        (lambda: lib.lbm_axi_init_vjp(p, None, None, 0, 8, p, None), "init_vjp"),
        (lambda: lib.lbm_axi_density(p, 8, -1, p, None), "density"),
        (lambda: lib.lbm_axi_ray_forward(p, -1, p, p, p, 2.0, 0.1, p, None), "ray_forward"),
        (lambda: lib.lbm_axi_ray_forward(p, 4, p, p, p, 1.0, 1.0, p, None), "ray_forward"),
        (lambda: lib.lbm_axi_ray_forward(p, 4, p, p, p, math.nan, 0.1, p, None), "ray_forward"),
        (lambda: lib.lbm_axi_ray_vjp(p, 4, p, p, p, p, 2.0, 0.1, 0, 8, p, None), "ray_vjp"),
        (lambda: lib.lbm_axi_ray_vjp(p, 4, p, p, p, p, 2.0, 0.1, 1 << 20, 1 << 12, p, None), "ray_vjp"),
        (lambda: lib.lbm_axi_ray_vjp(p, 4, p, p, p, p, 2.0, math.inf, 8, 8, p, None), "ray_vjp"),
        (lambda: lib.lbm_axi_ray_vjp(None, 4, p, p, p, p, 2.0, 0.1, 8, 8, p, None), "ray_vjp"),
        (lambda: lib.lbm_axi_misfit(p, p, -3, p, None, None), "misfit"),
        (lambda: lib.lbm_axi_misfit(p, None, 3, p, None, None), "misfit"),
    ]
    for call, name in cases:
        assert call() == L.EINVAL, name
        assert name in L.last_error(), (name, L.last_error())


def test_batch_rejects_midlink_source():
    from paper_1310_1871_amd import batch as B
    from paper_1310_1871_amd import lbm_axi as L
    ps = (L.Params * 2)(L.make_params(64, 32), L.make_params(64, 32, flags=L.FLAG_MIDLINK))
    assert B._lib.lbm_axi_batch_workspace_bytes(ps, 2) == 0
    assert "MIDLINK" in L.last_error()


def test_empty_batch_is_rejected():
    """A batch needs at least one instance: a count of 0 (or a NULL list)
    gives no workspace size and an error message."""
    from paper_1310_1871_amd import batch as B
    from paper_1310_1871_amd import lbm_axi as L
    ps = (L.Params * 1)(L.make_params(64, 32))
    assert B._lib.lbm_axi_batch_workspace_bytes(ps, 0) == 0
    assert "at least one instance" in L.last_error()
    assert B._lib.lbm_axi_batch_workspace_bytes(None, 1) == 0
    assert B._lib.lbm_axi_batch_workspace_bytes(ps, 1) > 0


def test_adjoint_size_limits():
    """The adjoint takes nz >= 4 and nr >= 6 (its psi window mirrors up to
    six rows at the axis and the wall) and one FP64 state below 4 GiB (its
    kernels' 32-bit byte offsets); other grids get no workspace size, and
    the calls return LBM_AXI_EINVAL before any device work."""
    from paper_1310_1871_amd import adjoint as A
    from paper_1310_1871_amd import lbm_axi as L
    ws = A._lib.lbm_axi_adjoint_workspace_bytes
    assert ws(4, 6) > 0 and ws(5, 8) > ws(4, 6)
    assert ws(3, 64) == 0 and ws(64, 5) == 0 and ws(1, 64) == 0
    # one FP64 state, 72 nz nr bytes, stays below 4 GiB (32-bit byte offsets):
    # 16383 x 3641 gives 4 294 836 216 bytes, one more row 4 296 015 792
    assert 72 * 16383 * 3641 < 2 ** 32 <= 72 * 16383 * 3642
    assert ws(16383, 3641) > 0 and ws(16383, 3642) == 0
    assert ws(1 << 20, 1 << 10) == 0  # within nz (nr + 12) < 2^31, beyond 4 GiB
    big = L.make_params(16383, 3642)
    rc = A._lib.lbm_axi_adjoint_step(ctypes.byref(big), ctypes.c_void_p(16), ctypes.c_void_p(16),
                                     ctypes.c_void_p(32), None, ctypes.c_void_p(16), 1 << 40, None)
    assert rc == L.EINVAL
    p = L.make_params(3, 64)
    dummy = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    rc = A._lib.lbm_axi_adjoint_step(ctypes.byref(p), dummy, dummy, ctypes.c_void_p(32), None, dummy, 1 << 20, None)
    assert rc == L.EINVAL


# The largest lattices accepted with nz = 16383 (= 129 x 127, ragged for
# the tiles): one population buffer, 9 planes of nz nr values each padded
# by 8 KiB, must stay below 4 GiB, the reach of the kernels' 32-bit buffer
# offsets.  9 (16383 x 3641 x 8 + 8192) = 4 294 909 944 bytes; one more row
# is 4 296 089 520.  FP32 storage holds twice the rows.
LARGEST_NZ = 16383
LARGEST_NR = {0: 3641, 1: 7282}


@pytest.mark.parametrize("precision", [0, 1])
def test_largest_accepted_lattice(precision):
    """check_params (no device) accepts the largest lattice of 16383
    columns and rejects one more row with a message; the workspace holds
    two buffers of at least 9 padded planes each."""
    from paper_1310_1871_amd import lbm_axi as L
    nr = LARGEST_NR[precision]
    size = 8 if precision == 0 else 4
    assert 9 * (LARGEST_NZ * nr * size + 8192) < 2 ** 32 <= 9 * (LARGEST_NZ * (nr + 1) * size + 8192)
    ok = L.make_params(LARGEST_NZ, nr, precision=precision, rho_ref=0.5 * precision)
    assert L.lib.lbm_axi_check_params(ctypes.byref(ok)) == L.OK
    assert L.workspace_bytes(ok) >= 2 * 9 * (LARGEST_NZ * nr * size + 8192)
    big = L.make_params(LARGEST_NZ, nr + 1, precision=precision, rho_ref=0.5 * precision)
    assert L.lib.lbm_axi_check_params(ctypes.byref(big)) == L.EINVAL
    assert "4 GiB" in L.last_error()
    assert L.workspace_bytes(big) == 0


def test_batch_binding_checks_its_lists():
    """The batch binding refuses initial densities that do not pair one to
    one with the instances' parameters (before any device work)."""
    from paper_1310_1871_amd import batch as B
    from paper_1310_1871_amd import lbm_axi as L
    with pytest.raises(ValueError):
        B.AxiBatch([L.make_params(64, 32), L.make_params(64, 32)], [None])
