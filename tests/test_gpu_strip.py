"""GPU parity of the row-marching step kernel (lbm_axi_set_kernel with
LBM_AXI_KERNEL_STRIP) against the CPU oracle, and against the tile kernel;
the tile kernel's other tile orders against its default order.

The strip computes the same step as the tile kernel (Sec. II: Eqs. scforce,
scAxisExtra, uhydro, ueq, condition_h, H_terms, lbm2d_mod_new and the
boundary rules of Sec. II.E) with a different organisation of the work:
a workgroup walks a 64-column band up a chunk of rows.  Chunk heights are
chosen so that chunks end mid-slab, at the axis and at the wall, and on
ragged lattices.  Bar: 1e-10 against the oracle (as the tile kernel's);
bitwise against the tile kernel in FP64 with the default options, where
both kernels evaluate every expression the same way."""
import numpy as np
import pytest
import torch

import oracle as O
from lbm_inputs import coexistence_densities, drop_density, random_state_fields, thread_density

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _lib():
    from paper_1310_1871_amd import lbm_axi as L
    return L


def _say(msg):
    print(msg, flush=True)


def _gpu(nz, nr, rho, steps, kind, rows=48, uz=None, ur=None, **kw):
    L = _lib()
    uz = np.zeros_like(rho) if uz is None else uz
    ur = np.zeros_like(rho) if ur is None else ur
    sim = L.AxiLBM(L.make_params(nz, nr, **kw), torch.from_numpy(rho).cuda(), torch.from_numpy(uz).cuda(),
                   torch.from_numpy(ur).cuda())
    sim.set_kernel(kind, rows)
    sim.step(steps)
    out = [t.cpu().numpy() for t in sim.moments()]
    f = sim.populations().cpu().numpy()
    sim.close()
    return out, f


def _parity(nz, nr, rho, steps, rows, uz=None, ur=None, **kw):
    L = _lib()
    _say(f"strip parity {nz}x{nr} steps={steps} chunk_rows={rows} {kw}")
    (rg, uzg, urg), _ = _gpu(nz, nr, rho, steps, L.KERNEL_STRIP, rows, uz, ur, **kw)
    p = O.make_params(nz, nr, **kw)
    z = np.zeros_like(rho)
    f = O.run(p, O.equilibrium(p, rho, z if uz is None else uz, z if ur is None else ur), steps)
    ro, uzo, uro = O.moments(p, f)
    assert np.isfinite(ro).all()
    err = (np.abs(rg - ro).max(), np.abs(uzg - uzo).max(), np.abs(urg - uro).max())
    _say(f"  max|drho|={err[0]:.3e} max|duz|={err[1]:.3e} max|dur|={err[2]:.3e}")
    assert max(err) <= TOL, err


@pytest.mark.parametrize("wall", [0, 1])
@pytest.mark.parametrize("rows", [7, 18, 64])
def test_strip_drop_1000_steps(wall, rows):
    """A deformed drop on 128 x 64 (one band pair, chunks of 7, 18 and 64
    rows), 1000 steps, both walls."""
    rg, rl = coexistence_densities(-5.5)
    rho = drop_density(128, 64, 64.0, 20.0, rl, rg, 2.0, {2: 3.0})
    _parity(128, 64, rho, 1000, rows, G=-5.5, tau=0.9, wall=wall)


@pytest.mark.parametrize("flags,wall", [(4, 0), (2, 1), (6, 0)])
def test_strip_options(flags, wall):
    """Guo forcing (4), the wall-derivative reading (2) and both (6)."""
    rg, rl = coexistence_densities(-5.0)
    rho = drop_density(128, 48, 64.0, 18.0, rl, rg, 2.0, {2: 2.0})
    _parity(128, 48, rho, 500, 20, G=-5.0, tau=0.9, wall=wall, flags=flags)


def test_strip_ragged_random_fields_body_force():
    """Random fields on a ragged 200 x 37 lattice (a partial last band and
    partial last chunk), planar and axisymmetric, body force."""
    rho, uz, ur = random_state_fields(11, 200, 37, rho_lo=0.5, rho_hi=1.5, u_amp=0.01)
    _parity(200, 37, rho, 300, 12, uz=uz, ur=ur, G=-4.0, tau=0.8, wall=0, gz=1e-5)
    _parity(200, 37, rho, 300, 37, uz=uz, ur=ur, G=-4.0, tau=0.8, wall=1, axisym=0)


def test_strip_large_ragged():
    """A ragged 4100 x 515 lattice through the row-marching kernel (chunks
    of 48 rows): 3 steps against the oracle on full fields."""
    rho, uz, ur = random_state_fields(4100515, 4100, 515, rho_lo=0.3, rho_hi=2.0, u_amp=0.01)
    _parity(4100, 515, rho, 3, 48, uz=uz, ur=ur, G=-5.0, tau=0.9, wall=1)


@pytest.mark.parametrize("precision", [0, 1])
def test_strip_matches_tile_kernel(precision):
    """The thread workload (4096 x 512), 100 steps, strip against tile
    kernel: bitwise in FP64, and within FP32 round-off growth (the two
    kernels contract the FP32 arithmetic differently) in FP32."""
    L = _lib()
    rg, rl = coexistence_densities(-5.5)
    rho = thread_density(4096, 512, 64.0, rl, rg, 2.0, 0.1, 1)
    kw = dict(G=-5.5, tau=0.8, wall=1, precision=precision, rho_ref=rg if precision else 0.0)
    _say(f"strip vs tile 4096x512 precision={precision}")
    _, fa = _gpu(4096, 512, rho, 100, L.KERNEL_TILE, **kw)
    _, fb = _gpu(4096, 512, rho, 100, L.KERNEL_STRIP, 48, **kw)
    d = np.abs(fa - fb).max()
    _say(f"  max |f_tile - f_strip| = {d:.3e}")
    if precision == 0:
        assert d == 0.0
    else:
        assert d < 1e-4


def test_strip_selection_rules():
    """set_kernel refuses lattices narrower than a band plus its halo and the
    options the strip does not have; open rows return to the tile kernel."""
    L = _lib()
    rho = np.ones((32, 64))
    sim = L.AxiLBM(L.make_params(64, 32, G=0.0), torch.from_numpy(rho).cuda())
    with pytest.raises(L.LbmAxiError) as e:
        sim.set_kernel(L.KERNEL_STRIP, 16)
    assert e.value.code == L.EUNSUP
    sim.close()
    rho = np.ones((32, 96))
    sim = L.AxiLBM(L.make_params(96, 32, G=0.0, flags=L.FLAG_MIDLINK), torch.from_numpy(rho).cuda())
    with pytest.raises(L.LbmAxiError) as e:
        sim.set_kernel(L.KERNEL_STRIP, 16)
    assert e.value.code == L.EUNSUP
    with pytest.raises(L.LbmAxiError):
        sim.set_kernel(L.KERNEL_STRIP, 0)
    sim.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("nz,nr", [(1024, 256), (4096, 512)])
def test_tile_orders_give_the_same_populations(precision, nz, nr):
    """LBM_AXI_KERNEL_TILE_ALTERNATE and LBM_AXI_KERNEL_TILE_COLUMNS only
    change the order in which the tiles run, LBM_AXI_KERNEL_TILE_PAIRS the
    nodes a thread holds and the width of its accesses: 21 steps (both buffer
    parities, graph replay included) give the default kernel's populations
    bit for bit.  Both lattices have whole tile rows per XCD, so the column
    order applies; node pairs apply to the larger one (64 x 16 tiles)."""
    L = _lib()
    rg, rl = coexistence_densities(-5.5)
    rho = thread_density(nz, nr, nr / 8.0, rl, rg, 2.0, 0.1, 1)
    kw = dict(G=-5.5, tau=0.8, wall=1, precision=precision, rho_ref=rg if precision else 0.0)
    _say(f"tile orders {nz}x{nr} precision={precision}")
    _, f0 = _gpu(nz, nr, rho, 21, L.KERNEL_TILE, **kw)
    for kind in (L.KERNEL_TILE_ALTERNATE, L.KERNEL_TILE_COLUMNS, L.KERNEL_TILE_PAIRS):
        _, fk = _gpu(nz, nr, rho, 21, kind, **kw)
        d = np.abs(f0 - fk).max()
        _say(f"  kind {kind}: max |f - f_default| = {d:.3e}")
        assert d == 0.0
