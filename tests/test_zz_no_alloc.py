"""The allocation-free reverse step (lbm_axi_adjoint_step_noalloc, scratch
in a static device array) against the workspace reverse step
(lbm_axi_adjoint_step) on the same inputs, through the C ABI: two calls in
a row on one GPU, the second on a smaller grid, each bitwise equal to the
workspace version (the same kernels on the same data); grids beyond the
static scratch are refused with LBM_AXI_ENOMEM before any device work."""
import ctypes

import numpy as np
import pytest
import torch

from lbm_inputs import coexistence_densities, drop_density, random_state_fields

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _libs():
    from paper_1310_1871_amd import adjoint as A
    from paper_1310_1871_amd import lbm_axi as L
    return L, A


def _inputs(nz, nr, seed):
    rg, rl = coexistence_densities(-5.5)
    rho = drop_density(nz, nr, nz / 2.0, 0.35 * nr, rl, rg, 2.0, {2: 0.05 * nr})
    _, uz, ur = random_state_fields(seed, nz, nr, u_amp=0.01)
    rng = np.random.Generator(np.random.PCG64(seed))
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]
    f = w * rho[None] * (1.0 + 0.01 * rng.uniform(-1, 1, size=(9, nr, nz)))
    lam = rng.standard_normal((9, nr, nz))
    return (torch.from_numpy(np.ascontiguousarray(f)).cuda(), torch.from_numpy(lam).cuda())


def _vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _both(nz, nr, seed):
    L, A = _libs()
    lib = A._lib
    lib.lbm_axi_adjoint_step_noalloc.restype = ctypes.c_int
    lib.lbm_axi_adjoint_step_noalloc.argtypes = [ctypes.POINTER(L.Params)] + [ctypes.c_void_p] * 5
    p = L.make_params(nz, nr, G=-5.5, tau=0.9, wall=0, axisym=1)
    f, lam_next = _inputs(nz, nr, seed)
    stream = torch.cuda.current_stream().cuda_stream
    # workspace version
    ws = torch.empty(lib.lbm_axi_adjoint_workspace_bytes(nz, nr) // 8, dtype=torch.float64, device="cuda")
    lam_ws = torch.empty_like(lam_next)
    g_ws = torch.zeros(2, dtype=torch.float64, device="cuda")
    rc = lib.lbm_axi_adjoint_step(ctypes.byref(p), _vp(f), _vp(lam_next), _vp(lam_ws), _vp(g_ws), _vp(ws),
                                  ws.numel() * 8, ctypes.c_void_p(stream))
    assert rc == L.OK
    # allocation-free version
    lam_na = torch.empty_like(lam_next)
    g_na = torch.zeros(2, dtype=torch.float64, device="cuda")
    rc = lib.lbm_axi_adjoint_step_noalloc(ctypes.byref(p), _vp(f), _vp(lam_next), _vp(lam_na), _vp(g_na),
                                          ctypes.c_void_p(stream))
    assert rc == L.OK, L.last_error()
    torch.cuda.synchronize()
    d_lam = (lam_na - lam_ws).abs().max().item()
    d_g = (g_na - g_ws).abs().max().item()
    _say(f"noalloc adjoint step {nz}x{nr}: max |dlam| = {d_lam:.3e}, max |dgrad| = {d_g:.3e}")
    assert torch.isfinite(lam_na).all()
    assert d_lam == 0.0 and d_g == 0.0
    return lam_na


def test_noalloc_adjoint_step_matches_workspace_step_twice():
    _both(768, 512, 31)   # first call on this GPU: looks the scratch up (16 x 16 tiles)
    _both(64, 32, 32)     # a smaller grid in the same scratch (16 x 8 tiles, the fused path)


def test_noalloc_rejects_grids_beyond_the_scratch():
    L, A = _libs()
    lib = A._lib
    lib.lbm_axi_adjoint_step_noalloc.restype = ctypes.c_int
    lib.lbm_axi_adjoint_step_noalloc.argtypes = [ctypes.POINTER(L.Params)] + [ctypes.c_void_p] * 5
    p = L.make_params(2048, 1024, G=-5.5, tau=0.9)
    dummy = ctypes.c_void_p(256)
    rc = lib.lbm_axi_adjoint_step_noalloc(ctypes.byref(p), dummy, dummy, dummy, None, None)
    assert rc == L.ENOMEM
    assert "static scratch" in L.last_error()
