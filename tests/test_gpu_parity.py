"""GPU parity of the FP64 HIP step against the CPU oracle (element by
element, same seeded inputs).  Bar: max |d rho|, max |d u| <= 1e-10 after
1000 steps at sizes the oracle runs in seconds, and on full fields at the
4096 x 512 bench size after a few steps; ragged and tiny grids included."""
import numpy as np
import pytest
import torch

import oracle as O
import oracle.diagnostics as D
from lbm_inputs import (coexistence_densities, drop_density, random_state_fields, static_drop,
                        thread_density)

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _lib():
    from paper_1310_1871_amd import lbm_axi as L
    return L


def _say(msg):
    print(msg, flush=True)


def _compare(nz, nr, rho, steps, G=-5.5, tau=1.0, wall=0, axisym=1, gz=0.0, uz=None, ur=None, tol=TOL, flags=0,
             kind=None):
    L = _lib()
    _say(f"parity case nz={nz} nr={nr} steps={steps} G={G} tau={tau} wall={wall} axisym={axisym} flags={flags}"
         f" kind={kind}")
    uz = np.zeros_like(rho) if uz is None else uz
    ur = np.zeros_like(rho) if ur is None else ur
    sim = L.AxiLBM(L.make_params(nz, nr, G=G, tau=tau, wall=wall, axisym=axisym, gz=gz, flags=flags),
                   torch.from_numpy(rho).cuda(), torch.from_numpy(uz).cuda(), torch.from_numpy(ur).cuda())
    if kind is not None:
        sim.set_kernel(kind)
    sim.step(steps)
    rg, uzg, urg = (t.cpu().numpy() for t in sim.moments())
    p = O.make_params(nz, nr, G=G, tau=tau, wall=wall, axisym=axisym, gz=gz, flags=flags)
    f = O.run(p, O.equilibrium(p, rho, uz, ur), steps)
    ro, uzo, uro = O.moments(p, f)
    assert np.isfinite(ro).all()
    err = (np.abs(rg - ro).max(), np.abs(uzg - uzo).max(), np.abs(urg - uro).max())
    _say(f"  max|drho|={err[0]:.3e} max|duz|={err[1]:.3e} max|dur|={err[2]:.3e}")
    assert max(err) <= tol, err
    return sim, f


@pytest.mark.parametrize("wall", [0, 1])
@pytest.mark.parametrize("axisym", [1, 0])
def test_static_drop_1000_steps(wall, axisym):
    """Static drop 64 x 32 (R = 10, rho 2.0/0.15, G = -5.5, tau = 1)."""
    c = static_drop()
    _compare(c.nz, c.nr, c.rho, 1000, G=c.G, tau=c.tau, wall=wall, axisym=axisym)


@pytest.mark.parametrize("wall", [0, 1])
def test_guo_forcing_static_drop_1000_steps(wall):
    """The Guo forcing option (the scheme the paper compares against in
    Sec. IV.A) on the static drop, both walls, against the oracle's."""
    c = static_drop()
    _compare(c.nz, c.nr, c.rho, 1000, G=c.G, tau=c.tau, wall=wall, flags=4)


def test_guo_forcing_ragged_and_body_force():
    """Guo forcing on a ragged grid with random fields and a body force."""
    nz, nr = 100, 37
    rho, uz, ur = random_state_fields(7337, nz, nr, rho_lo=0.5, rho_hi=1.5, u_amp=0.01)
    _compare(nz, nr, rho, 200, G=-4.0, tau=0.8, wall=0, gz=1e-5, uz=uz, ur=ur, flags=4)


@pytest.mark.parametrize("flags", [2, 6])
@pytest.mark.parametrize("wall", [0, 1])
def test_wall_derivative_option_static_drop(wall, flags):
    """The other reading of the wall derivative rule (flag 2), alone and
    with Guo forcing (flag 6), on a drop that touches the wall region:
    512 steps against the oracle."""
    from lbm_inputs import drop_density
    rg, rl = coexistence_densities(-5.0)
    rho = drop_density(64, 24, 32.0, 14.0, rl, rg, 2.0, {2: 1.5})
    _compare(64, 24, rho, 512, G=-5.0, tau=0.9, wall=wall, flags=flags)


def test_wall_derivative_option_large_tiles():
    """Flag 2 on the large 64 x 16 tile shape (ragged 4100 x 515), 4 steps."""
    nz, nr = 4100, 515
    rho, uz, ur = random_state_fields(4100516, nz, nr, rho_lo=0.3, rho_hi=2.0, u_amp=0.01)
    _compare(nz, nr, rho, 4, G=-5.0, tau=0.9, wall=0, uz=uz, ur=ur, flags=2)


@pytest.mark.parametrize("flags", [16, 16 | 4, 16 | 2])
@pytest.mark.parametrize("wall", [0, 1])
def test_midlink_source_static_drop(wall, flags):
    """The mid-link reading of the source (flag 16: a moments pass writes H
    and the mass source, the step averages h_i over each link), alone, with
    Guo forcing and with the wall-derivative reading: 500 steps."""
    from lbm_inputs import drop_density
    rg, rl = coexistence_densities(-5.0)
    rho = drop_density(64, 24, 32.0, 14.0, rl, rg, 2.0, {2: 1.5})
    _compare(64, 24, rho, 500, G=-5.0, tau=0.9, wall=wall, flags=flags)


def test_midlink_source_ragged_fields_and_large_tiles():
    """Flag 16 with random fields and a body force on a ragged small-tile
    grid (200 steps), and on the large 64 x 16 tile shape (ragged 4100 x 515, 3
    steps)."""
    rho, uz, ur = random_state_fields(1616, 100, 37, rho_lo=0.5, rho_hi=1.5, u_amp=0.01)
    _compare(100, 37, rho, 200, G=-4.0, tau=0.8, wall=0, gz=1e-5, uz=uz, ur=ur, flags=16)
    rho, uz, ur = random_state_fields(4100517, 4100, 515, rho_lo=0.3, rho_hi=2.0, u_amp=0.01)
    _compare(4100, 515, rho, 3, G=-5.0, tau=0.9, wall=1, uz=uz, ur=ur, flags=16)


def test_oscillating_drop_shape_1000_steps():
    """Drop oscillation lattice 256 x 128 (P2 perturbation, seeded noise),
    tau = 0.8 (the lowest tau of that workload the scheme keeps stable)."""
    from lbm_inputs import oscillating_drop
    c = oscillating_drop(tau=0.8)
    _compare(c.nz, c.nr, c.rho, 1000, G=c.G, tau=c.tau, wall=c.wall)


@pytest.mark.parametrize("nz,nr", [(100, 37), (65, 17), (130, 22), (7, 6), (1, 64), (70, 6)])
def test_ragged_and_tiny_grids(nz, nr):
    """Grids that are not multiples of the 64 x 16 tile, a single column
    (the Table I lattice), the minimum radial size, and a 7-wide periodic
    strip whose stencils wrap several times."""
    rho, uz, ur = random_state_fields(nz * 1000 + nr, nz, nr, rho_lo=0.5, rho_hi=1.5, u_amp=0.01)
    _compare(nz, nr, rho, 200, G=-4.0, tau=0.9, wall=1, uz=uz, ur=ur)


@pytest.mark.parametrize("G,tau,lo,hi", [(0.0, 0.51, 0.95, 1.05), (-4.0, 1.5, 0.7, 1.3)])
def test_extreme_relaxation_times(G, tau, lo, hi):
    """The ends of the relaxation times the scheme runs: tau = 0.51 (nu =
    0.0033, 1/tau near 2) single phase, and tau = 1.5 (nu = 1/3, the
    viscous axisymmetric source terms large) with the SC force; random
    fields with velocity on the ragged 100 x 37 grid, 200 steps against the
    oracle."""
    rho, uz, ur = random_state_fields(int(tau * 100), 100, 37, rho_lo=lo, rho_hi=hi, u_amp=0.02)
    _compare(100, 37, rho, 200, G=G, tau=tau, wall=1, uz=uz, ur=ur)


def test_pipe_flow_body_force():
    """Single phase with the body force (Hagen–Poiseuille set-up, 16 x 16)."""
    rho = np.ones((16, 16))
    _compare(16, 16, rho, 1000, G=0.0, tau=1.0, wall=0, gz=1e-5)


def test_full_size_thread_fields():
    """Rayleigh–Plateau thread at the bench size 4096 x 512, tau = 0.8, in
    the launch configuration the benchmark times: full fields after 3 steps."""
    G = -5.5
    rg, rl = coexistence_densities(G)
    rho = thread_density(4096, 512, 64.0, rl, rg, 2.0, 0.1, 1)
    _compare(4096, 512, rho, 3, G=G, tau=0.8, wall=1)


@pytest.mark.parametrize("precision", [0, 1])
def test_largest_lattice_repeats_one_period(precision):
    """The largest lattice the library accepts with nz = 16383: each
    population buffer just below 4 GiB (3641 rows in FP64, 7282 in FP32),
    the end of the kernels' 32-bit buffer offsets, and ragged for the tiles
    (the last tile column 63 wide, the last tile row 9 or 2 rows).  Its
    state repeats with period 127 in z (129 periods).  z is periodic, so the
    step commutes with the shift by one period: after 12 steps every
    population of the large lattice equals the one of a 127-column lattice
    run alone (small tiles), which in FP64 matches the oracle.  The two tile
    shapes order a few operations differently, so "equals" is up to the
    storage type's rounding (measured 5.6e-16 in FP64, 3.6e-7 in FP32);
    a wrapped offset or a misplaced plane anywhere in the 4 GiB gives
    differences of the populations' own size.  The 3D mass of the large
    lattice is 129 times the small one's: to summation order in FP64, and
    in FP32 to roundings of random sign in 1.2e8 nodes (measured 2.7e-11,
    bound 1e-9)."""
    L = _lib()
    nz, period = 16383, 127
    nr = 3641 if precision == 0 else 7282
    steps, G, tau, wall = 12, -5.0, 0.9, precision
    rref = 0.0 if precision == 0 else 0.5
    _say(f"largest lattice case precision={precision} nz={nz} nr={nr} period={period} steps={steps}")
    rho, uz, ur = random_state_fields(16383 + precision, period, nr, rho_lo=0.3, rho_hi=2.0, u_amp=0.01)

    def run(n, reps):
        p = L.make_params(n, nr, G=G, tau=tau, wall=wall, precision=precision, rho_ref=rref)
        dev = [torch.from_numpy(a).cuda().repeat(1, reps) for a in (rho, uz, ur)]
        sim = L.AxiLBM(p, *dev)
        sim.step(steps)
        return sim

    small = run(period, 1)
    dt = torch.float64 if precision == 0 else torch.float32
    fs = small.get_state().view(dt).reshape(9, nr, 1, period)
    mass_small = small.reduce()[0]
    big = run(nz, nz // period)
    fb = big.get_state().view(dt).reshape(9, nr, nz // period, period)
    mass_big = big.reduce()[0]
    torch.cuda.synchronize()
    err = max((fb[i] - fs[i]).abs().max().item() for i in range(9))
    _say(f"  max |f_large - f_period| = {err:.3e}; 3D mass {mass_big!r} against 129 x {mass_small!r}")
    del fb
    big.close()
    assert err <= (1e-12 if precision == 0 else 1e-5)
    assert abs(mass_big - (nz // period) * mass_small) <= (1e-12 if precision == 0 else 1e-9) * abs(mass_big)
    if precision == 0:
        rg, uzg, urg = (t.cpu().numpy() for t in small.moments())
        p = O.make_params(period, nr, G=G, tau=tau, wall=wall)
        ro, uzo, uro = O.moments(p, O.run(p, O.equilibrium(p, rho, uz, ur), steps))
        e = max(np.abs(rg - ro).max(), np.abs(uzg - uzo).max(), np.abs(urg - uro).max())
        _say(f"  period lattice against the oracle: {e:.3e}")
        assert e <= TOL
    small.close()


@pytest.mark.parametrize("wall", [0, 1])
def test_large_tile_shape_ragged(wall):
    """A lattice large enough for the large 64 x 16 tiles (2145 of them) but
    not a multiple of them: 4100 x 515 leaves a last tile column 4 wide and a
    last tile row with 3 real rows, so the ghost rows beyond the wall fill most
    of its velocity window.  Both wall rules, random smooth fields, 6 steps
    against the oracle."""
    nz, nr = 4100, 515
    rho, uz, ur = random_state_fields(4100515 + wall, nz, nr, rho_lo=0.3, rho_hi=2.0, u_amp=0.01)
    _compare(nz, nr, rho, 6, G=-5.0, tau=0.9, wall=wall, uz=uz, ur=ur)


@pytest.mark.parametrize("nz,nr", [(65536, 6), (1, 16390)])
def test_large_tiles_on_degenerate_shapes(nz, nr):
    """Lattices that take the large 64 x 16 tiles (1024 or more of them)
    in degenerate shapes: 65536 x 6, one tile row that is both the axis
    and the wall tile with 6 of its 16 rows real; 1 x 16390, a single
    column, so every tile's window wraps z many times (the narrow-lattice
    path of the periodic wrap), ragged in r.  Random fields, 20 steps
    against the oracle."""
    rho, uz, ur = random_state_fields(nz + nr, nz, nr, rho_lo=0.6, rho_hi=1.4, u_amp=0.01)
    _compare(nz, nr, rho, 20, G=-4.0, tau=0.9, wall=1, uz=uz, ur=ur)


@pytest.mark.parametrize("nz,nr,flags,wall", [(4100, 515, 0, 0), (4100, 515, 4 | 2, 1), (2049, 520, 0, 1),
                                              (2048, 520, 8, 1), (4098, 515, 16, 0)])
def test_node_pair_kernel(nz, nr, flags, wall):
    """LBM_AXI_KERNEL_TILE_PAIRS: each thread holds two z-adjacent nodes of
    a 64 x 16 tile and moves them in one access per plane where nz is even
    and z periodic.  Even ragged lattices with the Guo and wall-derivative
    options and with the mid-link source take the paired accesses; odd nz
    and z walls (whose mirror reverses a pair) take one access per node.
    4 steps against the oracle, and the populations equal the default tile
    kernel's bit for bit."""
    L = _lib()
    rho, uz, ur = random_state_fields(nz * 7 + nr + flags, nz, nr, rho_lo=0.5, rho_hi=1.5, u_amp=0.01)
    sim, _ = _compare(nz, nr, rho, 4, G=-4.0, tau=0.9, wall=wall, uz=uz, ur=ur, flags=flags,
                      kind=L.KERNEL_TILE_PAIRS)
    fp = sim.populations().cpu().numpy()
    sim.close()
    ref = L.AxiLBM(L.make_params(nz, nr, G=-4.0, tau=0.9, wall=wall, flags=flags), torch.from_numpy(rho).cuda(),
                   torch.from_numpy(uz).cuda(), torch.from_numpy(ur).cuda())
    ref.step(4)
    d = np.abs(ref.populations().cpu().numpy() - fp).max()
    ref.close()
    _say(f"  max |f_pairs - f_tile| = {d:.3e}")
    assert d == 0.0


def test_reduce_and_moments_match_oracle_diagnostics():
    L = _lib()
    c = static_drop()
    _say("reduce case static drop 64x32, 300 steps")
    sim = L.AxiLBM(L.make_params(c.nz, c.nr, G=c.G, tau=c.tau), torch.from_numpy(c.rho).cuda())
    sim.step(300)
    red = sim.reduce()
    p = O.make_params(c.nz, c.nr, G=c.G, tau=c.tau)
    ro, uzo, uro = O.moments(p, O.run(p, O.equilibrium(p, c.rho, 0 * c.rho, 0 * c.rho), 300))
    ref = [D.mass_3d(ro), D.momentum_z_3d(ro, uzo), D.kinetic_energy(ro, uzo, uro), D.mass_2d(ro)]
    for a, b in zip(red, ref):
        assert abs(a - b) <= 1e-10 * max(1.0, abs(b)), (red, ref)


@pytest.mark.parametrize("case", ["drop", "thread"])
def test_interface_diagnostics_match_oracle(case):
    """lbm_axi_interface against the oracle's diagnostics on the oracle's
    state after the same steps: the drop intercept A(t), the radius profile
    R(z) with its minimum (thread neck) and maximum, the minimum density on
    the row next to the axis (break-up), and the Laplace pressure jump."""
    L = _lib()
    if case == "drop":
        c = static_drop()
        nz, nr, rho, G, tau, steps = c.nz, c.nr, c.rho, c.G, c.tau, 300
        mid = 0.5 * (c.rho_l + c.rho_g)
    else:
        G, tau, nz, nr, steps = -5.5, 1.0, 512, 96, 200
        rg, rl = coexistence_densities(G)
        rho = thread_density(nz, nr, 24.0, rl, rg, 2.0, 0.2, 2)
        mid = 0.5 * (rl + rg)
    _say(f"interface diagnostics {case} {nz}x{nr}, {steps} steps")
    sim = L.AxiLBM(L.make_params(nz, nr, G=G, tau=tau, wall=1), torch.from_numpy(rho).cuda())
    sim.step(steps)
    radius = torch.empty(nz, dtype=torch.float64, device="cuda")
    got = sim.interface(mid, nz // 2, radius)
    sim.close()
    p = O.make_params(nz, nr, G=G, tau=tau, wall=1)
    ro, _, _ = O.moments(p, O.run(p, O.equilibrium(p, rho, 0 * rho, 0 * rho), steps))
    prof = np.array([D.axis_intercept(ro, z, mid) for z in range(nz)])
    assert np.abs(radius.cpu().numpy() - prof).max() < 1e-9
    want = {"A": prof[nz // 2], "neck": prof.min(), "r_max": prof.max(), "rho_axis_min": ro[0].min(),
            "rho_in": ro[0, nz // 2], "rho_out": ro[-1, 0],
            "dp": D.pressure(ro[0, nz // 2], G) - D.pressure(ro[-1, 0], G)}
    for k, v in want.items():
        assert abs(got[k] - v) < 1e-9 * max(1.0, abs(v)), (k, got[k], v)


def test_state_roundtrip_and_resume():
    """get_state/set_state: a run checkpointed at step 100 and resumed
    reproduces the uninterrupted run bit for bit."""
    L = _lib()
    c = static_drop()
    _say("checkpoint case static drop 64x32")
    a = L.AxiLBM(L.make_params(c.nz, c.nr, G=c.G, tau=c.tau), torch.from_numpy(c.rho).cuda())
    a.step(100)
    ck = a.get_state()
    a.step(150)
    fa = a.populations()
    b = L.AxiLBM(L.make_params(c.nz, c.nr, G=c.G, tau=c.tau), torch.from_numpy(c.rho * 0 + 1.0).cuda())
    b.set_state(ck)
    b.step(150)
    assert torch.equal(fa, b.populations())


@pytest.mark.parametrize("fp32", [False, True])
def test_padded_buffers_keep_the_plain_state_layout(fp32):
    """The library pads every population plane of its own buffers; the
    caller sees the plain [9][nr][nz] layout.  On a ragged 4100 x 515
    lattice: a state set and read back is unchanged bit for bit; a record of
    3 states starts with that state, and its last state is the handle's
    state afterwards; a step on the handle equals a step in the record."""
    L = _lib()
    nz, nr = 4100, 515
    rho, uz, ur = random_state_fields(515, nz, nr, rho_lo=0.5, rho_hi=1.5, u_amp=0.01)
    p = L.make_params(nz, nr, G=-4.0, tau=0.9, wall=1, precision=L.FP32_SHIFTED if fp32 else L.FP64,
                      rho_ref=0.5 if fp32 else 0.0)
    _say(f"padded layout round trip {nz}x{nr} fp32={fp32}")
    sim = L.AxiLBM(p, torch.from_numpy(rho).cuda(), torch.from_numpy(uz).cuda(), torch.from_numpy(ur).cuda())
    sim.step(2)
    s0 = sim.get_state()
    gen = torch.Generator(device="cuda").manual_seed(7)
    noise = torch.rand(s0.numel() // (4 if fp32 else 8), generator=gen, device="cuda",
                       dtype=torch.float32 if fp32 else torch.float64) * 1e-3
    st = (s0.view(noise.dtype) + noise).view(torch.uint8)
    sim.set_state(st)
    assert torch.equal(sim.get_state(), st)
    rec = torch.empty(3 * st.numel(), dtype=torch.uint8, device="cuda")
    sim.record(3, rec)
    n = st.numel()
    assert torch.equal(rec[:n], st)
    assert torch.equal(sim.get_state(), rec[2 * n:])
    sim.set_state(rec[n:2 * n])
    sim.step(1)
    assert torch.equal(sim.get_state(), rec[2 * n:])
    sim.close()


@pytest.mark.parametrize("rho_val", [0.1, 2.3])
@pytest.mark.parametrize("wall", [0, 1])
def test_rest_state_invariant_on_gpu(wall, rho_val):
    """Uniform density at rest stays W_i rho.  The densities are outside the
    spinodal region of G = -5.5 (dp/drho > 0), where a uniform state is
    mechanically stable; inside it, round-off residuals of the stencils
    grow exponentially by design of the model."""
    L = _lib()
    rho = np.full((24, 70), rho_val)
    _say(f"rest state 70x24 wall={wall} rho={rho_val}")
    sim = L.AxiLBM(L.make_params(70, 24, G=-5.5, tau=0.8, wall=wall), torch.from_numpy(rho).cuda())
    f0 = sim.populations()
    sim.step(500)
    assert (sim.populations() - f0).abs().max().item() < 1e-12


def test_nonfinite_is_reported():
    """A NaN-seeded density makes the FP64 reduction report ENONFINITE."""
    L = _lib()
    rho = np.full((16, 64), 1.0)
    rho[3, 5] = np.nan
    _say("non-finite case")
    sim = L.AxiLBM(L.make_params(64, 16, G=0.0, tau=1.0), torch.from_numpy(rho).cuda())
    with pytest.raises(L.LbmAxiError) as e:
        sim.reduce()
    assert e.value.code == L.ENONFINITE


@pytest.mark.parametrize("precision", [0, 1])
def test_populations_export_decodes_on_device(precision):
    """lbm_axi_populations returns f_i in FP64: the stored state itself in
    FP64 storage (bit for bit), and the FP32 values plus W_i rho_ref (added
    in double) in shifted storage, equal to a decode of get_state done here
    up to the rounding of that one multiply-add (the device may fuse it)."""
    L = _lib()
    rg, rl = coexistence_densities(-5.5)
    rho = drop_density(96, 48, 48.0, 14.0, rl, rg, 2.0, {2: 1.0})
    rref = 0.0 if precision == 0 else rg
    sim = L.AxiLBM(L.make_params(96, 48, G=-5.5, tau=0.9, precision=precision, rho_ref=rref),
                   torch.from_numpy(rho).cuda())
    sim.step(20)
    f = sim.populations().cpu().numpy()
    raw = sim.get_state().cpu().numpy()
    if precision == 0:
        assert np.array_equal(f, raw.view(np.float64).reshape(9, 48, 96))
    else:
        w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
        ref = raw.view(np.float32).reshape(9, 48, 96).astype(np.float64) + w[:, None, None] * rref
        assert np.abs(f - ref).max() <= 2.0 ** -52 * np.abs(ref).max()
    sim.close()


def test_fp32_global_sums_are_fp64():
    """In FP32 storage the 3D mass and 2D mass of lbm_axi_reduce are FP64
    sums of the decoded populations: they equal a numpy FP64 sum of
    lbm_axi_populations to summation-order round-off (1e-14)."""
    L = _lib()
    rg, rl = coexistence_densities(-5.5)
    rho = drop_density(256, 128, 128.0, 40.0, rl, rg, 2.0, {2: 2.0})
    sim = L.AxiLBM(L.make_params(256, 128, G=-5.5, tau=0.9, precision=L.FP32_SHIFTED, rho_ref=rg),
                   torch.from_numpy(rho).cuda())
    sim.step(50)
    red = sim.reduce()
    f = sim.populations().cpu().numpy()
    dens = f.sum(axis=0)
    r = np.arange(128)[:, None] + 0.5
    m3 = float(np.sum(2.0 * np.pi * r * dens))
    _say(f"FP32 3D mass: reduce {red[0]!r} numpy {m3!r}")
    assert abs(red[0] - m3) <= 1e-14 * m3
    assert abs(red[3] - float(dens.sum())) <= 1e-14 * float(dens.sum())
    rg_, _, _ = (t.cpu().numpy() for t in sim.moments())
    assert np.abs(rg_ - dens).max() <= 1e-14
    sim.close()


def test_stability_warning_on_create():
    """G < -6 (outside the rule of thumb of Sec. II.D) creates the handle
    with LBM_AXI_WARN_STABILITY, which the binding turns into a warning;
    the lattice still steps."""
    L = _lib()
    rho = np.full((32, 64), 1.0)
    with pytest.warns(L.StabilityWarning):
        sim = L.AxiLBM(L.make_params(64, 32, G=-6.5, tau=1.0), torch.from_numpy(rho).cuda())
    sim.step(5)
    assert np.isfinite(sim.reduce()).all()
    with pytest.warns(L.StabilityWarning):
        sim.set_coupling(-6.2, 1.0)
    sim.close()


def test_graph_replay_matches_direct_launches():
    """On a stream other than the null stream, lbm_axi_step replays pairs of
    steps of a small lattice as a captured graph.  After each of several
    calls (odd and even step counts, eager work between them, a change of G
    and tau that drops the graphs) the state equals that of direct launches
    on the null stream bit for bit."""
    L = _lib()
    rg, rl = coexistence_densities(-5.5)
    rho = drop_density(128, 64, 64.0, 20.0, rl, rg, 2.0, {2: 3.0})
    side = torch.cuda.Stream()
    p = L.make_params(128, 64, G=-5.5, tau=0.9)
    a = L.AxiLBM(p, torch.from_numpy(rho).cuda(), stream=side)
    b = L.AxiLBM(L.make_params(128, 64, G=-5.5, tau=0.9), torch.from_numpy(rho).cuda())
    torch.cuda.synchronize()
    for n, coupling in ((7, None), (10, None), (4, (-5.2, 1.0)), (13, None), (2, None)):
        if coupling:
            a.set_coupling(*coupling)
            b.set_coupling(*coupling)
        a.step(n)
        b.step(n)
        ra, rb = a.reduce(), b.reduce()  # eager work between the replays (synchronises)
        side.synchronize()
        fa = a.populations()
        side.synchronize()
        fb = b.populations()
        torch.cuda.synchronize()
        _say(f"graph replay {n} steps: max |df| = {(fa - fb).abs().max().item():.3e}")
        assert torch.equal(fa, fb) and ra == rb
    a.close()
    b.close()


def test_zero_counts_change_nothing_and_negative_counts_fail():
    """Empty work: lbm_axi_step(0), lbm_axi_batch_step(0) and
    lbm_axi_adjoint_run with k = 0 return OK and leave every state (and the
    adjoint's lam and gradient sums) bit for bit as it was; the steps after
    them match a lattice that never made the empty call.  A negative count,
    and a record of 0 states, fail with LBM_AXI_EINVAL."""
    import ctypes
    from paper_1310_1871_amd import adjoint as A
    from paper_1310_1871_amd import batch as B
    L = _lib()
    nz, nr = 100, 37
    rho, uz, ur = random_state_fields(10037, nz, nr, rho_lo=0.5, rho_hi=1.5, u_amp=0.01)
    _say("zero-count case single lattice 100x37")
    p = L.make_params(nz, nr, G=-4.0, tau=0.9, wall=1)
    fields = [torch.from_numpy(a).cuda() for a in (rho, uz, ur)]
    a = L.AxiLBM(p, *fields)
    b = L.AxiLBM(L.make_params(nz, nr, G=-4.0, tau=0.9, wall=1), *fields)
    a.step(3)
    b.step(3)
    before = a.populations()
    assert L.lib.lbm_axi_step(a._h, 0) == L.OK
    assert torch.equal(a.populations(), before)
    assert L.lib.lbm_axi_step(a._h, -1) == L.EINVAL and ">= 0" in L.last_error()
    rec = torch.empty(a.state_bytes(), dtype=torch.uint8, device="cuda")
    assert L.lib.lbm_axi_record(a._h, 0, ctypes.c_void_p(rec.data_ptr())) == L.EINVAL
    a.step(5)
    b.step(5)
    assert torch.equal(a.populations(), b.populations())
    f_state = a.get_state().view(torch.float64).reshape(9, nr, nz).clone()
    a.close()
    b.close()

    _say("zero-count case batch of two")
    ps = [L.make_params(64, 32, G=-5.0, tau=0.9), L.make_params(nz, nr, G=-4.0, tau=0.9, wall=1)]
    rg, rl = coexistence_densities(-5.0)
    rhos = [torch.from_numpy(drop_density(64, 32, 32.0, 10.0, rl, rg, 2.0, {2: 1.0})).cuda(), fields[0]]
    bat = B.AxiBatch(ps, rhos)
    bat.step(2)
    bat.synchronize()
    keep = [bat.populations(k) for k in range(2)]
    assert B._lib.lbm_axi_batch_step(bat._h, 0) == L.OK
    assert B._lib.lbm_axi_batch_step(bat._h, -2) == L.EINVAL
    bat.synchronize()
    assert all(torch.equal(bat.populations(k), keep[k]) for k in range(2))
    bat.close()

    _say("zero-count case adjoint run")
    dev = torch.device("cuda")
    ws = torch.empty(A._lib.lbm_axi_adjoint_workspace_bytes(nz, nr) // 8, dtype=torch.float64, device=dev)
    lam = torch.from_numpy(np.random.Generator(np.random.PCG64(5)).standard_normal((9, nr, nz))).to(dev)
    lam0 = lam.clone()
    acc = torch.tensor([0.25, -0.5], dtype=torch.float64, device=dev)
    A.adjoint_run(p, f_state, 0, lam, torch.empty_like(lam), acc, ws)
    torch.cuda.synchronize()
    assert torch.equal(lam, lam0)
    assert acc.tolist() == [0.25, -0.5]


def test_own_stream_handle_orders_caller_tensors():
    """A handle with a stream of its own, used with no explicit
    synchronisation: the initial density is computed on the caller's stream
    just before create, the state is replaced from a tensor the caller has
    just written, and moments, populations and get_state are reduced on the
    caller's stream as soon as they return, then freed, in a loop (so the
    allocator hands their memory to the next call at once).  Every value
    equals that of a handle on the caller's stream, bit for bit; the
    binding orders the two streams around each call that touches caller
    memory."""
    L = _lib()
    nz, nr = 128, 64
    rho_np, uz_np, ur_np = random_state_fields(12864, nz, nr, rho_lo=0.5, rho_hi=1.5, u_amp=0.01)
    _say("own-stream handle case 128x64")
    side = torch.cuda.Stream()
    base = torch.from_numpy(rho_np).cuda()
    ref = L.AxiLBM(L.make_params(nz, nr, G=-4.0, tau=0.9), base)
    a = L.AxiLBM(L.make_params(nz, nr, G=-4.0, tau=0.9), base * 1.0, stream=side)
    sums_ref, sums = [], []
    for it in range(6):
        ref.step(7)
        a.step(7)
        for sim, acc in ((ref, sums_ref), (a, sums)):
            rho, uz, ur = sim.moments()
            acc.append(torch.stack([rho.sum(), uz.abs().sum(), ur.abs().sum()]))
            del rho, uz, ur
            acc.append(sim.populations().sum(dim=(1, 2)))
            acc.append(sim.get_state().view(torch.float64).reshape(9, nr, nz)[:, ::7, ::5].sum(dim=(1, 2)))
        if it == 3:
            # both lattices continue from one state written on the caller's stream
            st = ref.get_state().view(torch.float64).reshape(9, nr, nz) * 1.0
            ref.set_state(st.reshape(-1).view(torch.uint8))
            a.set_state((st * 1.0).reshape(-1).view(torch.uint8))
            del st
    got = torch.cat(sums).cpu()
    want = torch.cat(sums_ref).cpu()
    _say(f"  max |difference| over {got.numel()} sums: {(got - want).abs().max().item():.3e}")
    assert torch.equal(got, want)
    a.close()
    ref.close()


def test_step_captured_into_a_caller_graph():
    """lbm_axi_step on a stream the caller captures (torch.cuda.graph):
    the step kernels go into the caller's graph instead of a graph of the
    library's own, an odd step count is refused there (the buffer parity
    is host state), and each of several replays, with eager work and a
    synchronisation between them, equals eager steps of a second lattice
    bit for bit.  The capture itself runs nothing."""
    L = _lib()
    rg, rl = coexistence_densities(-5.5)
    rho = drop_density(128, 64, 64.0, 20.0, rl, rg, 2.0, {2: 3.0})
    _say("caller graph capture of lbm_axi_step 128x64")
    a = L.AxiLBM(L.make_params(128, 64, G=-5.5, tau=0.9), torch.from_numpy(rho).cuda())
    b = L.AxiLBM(L.make_params(128, 64, G=-5.5, tau=0.9), torch.from_numpy(rho).cuda())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        with pytest.raises(L.LbmAxiError) as e:
            a.step(3)
        a.step(6)
    assert e.value.code == L.EINVAL and "even" in str(e.value)
    torch.cuda.synchronize()
    assert torch.equal(a.populations(), b.populations())
    for rep in range(4):
        g.replay()
        b.step(6)
        ra, rb = a.reduce(), b.reduce()  # eager work between the replays (synchronises)
        fa, fb = a.populations(), b.populations()
        _say(f"  replay {rep}: max |df| = {(fa - fb).abs().max().item():.3e}")
        assert torch.equal(fa, fb) and ra == rb, rep
    a.close()
    b.close()
