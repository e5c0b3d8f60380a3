"""Pins of the oracle's FP64 diagnostics against closed forms and physical
invariants (not against their own formulas)."""
import numpy as np
import pytest

import oracle as O
import oracle.diagnostics as D
from lbm_inputs import coexistence_densities, drop_density, legendre, node_coords, tanh_profile


def test_3d_integrals_of_uniform_fields():
    """With r_j = j + 1/2 (Sec. III, nodes half a spacing off the axis),
    sum_j 2 pi r_j = pi nr^2 exactly: the 3D mass of a uniform density is
    rho pi nr^2 nz, the volume of the cylinder of radius nr and length nz.
    Momentum and kinetic energy follow with u uniform."""
    nz, nr, rho, uz, ur = 7, 13, 1.7, 0.03, -0.01
    r = np.full((nr, nz), rho)
    assert D.mass_3d(r) == pytest.approx(rho * np.pi * nr * nr * nz, rel=1e-14)
    assert D.mass_2d(r) == pytest.approx(rho * nr * nz, rel=1e-14)
    assert D.momentum_z_3d(r, np.full_like(r, uz)) == pytest.approx(rho * uz * np.pi * nr * nr * nz, rel=1e-14)
    ke = D.kinetic_energy(r, np.full_like(r, uz), np.full_like(r, ur))
    assert ke == pytest.approx(0.5 * rho * (uz * uz + ur * ur) * np.pi * nr * nr * nz, rel=1e-14)


def test_equivalent_radius_of_a_sphere():
    """A diffuse sphere of radius R on the axis has the 3D liquid volume of
    (4/3) pi R^3 up to the quadrature of the tanh profile: R_eq within 1 %."""
    nz, nr, R = 96, 48, 20.0
    rho = drop_density(nz, nr, nz / 2.0, R, 2.0, 0.1, 1.5)
    assert D.equivalent_radius(rho, 2.0, 0.1) == pytest.approx(R, rel=0.01)


def test_axis_intercept_linear_profile():
    """A column whose density falls linearly through rho_mid between two
    nodes: the intercept is the exact crossing point."""
    nr = 20
    r = np.arange(nr) + 0.5
    col = 2.0 - 0.1 * r  # crosses 1.0 at r = 10
    rho = np.repeat(col[:, None], 3, axis=1)
    assert D.axis_intercept(rho, 1, 1.0) == pytest.approx(10.0, abs=1e-12)


def test_interface_radius_linear_in_z():
    """For phi linear in z the bilinear interpolant is exact, so the ray sum
    has the closed form (a + b zc) n ds + b cos(theta) (n ds)^2 / 2 with
    n = floor(s_max / ds) midpoint samples."""
    nz, nr, zc = 64, 40, 32.0
    a, b = 0.3, 0.01
    z, _ = node_coords(nz, nr)
    rho_l, rho_g = 1.0, 0.0
    rho = a + b * z
    th = [0.3, 1.2, 2.5]
    W = D.interface_radius_weights(nz, nr, zc, th, ds=0.5)
    got = D.interface_radius(rho, W, rho_l, rho_g)
    s_max = min(nz / 2.0, float(nr)) - 1.0
    n = int(np.floor(s_max / 0.5))
    L = n * 0.5
    want = [(a + b * zc) * L + b * np.cos(t) * L * L / 2.0 for t in th]
    assert np.allclose(got, want, rtol=0, atol=1e-12)


def test_interface_radius_of_a_perturbed_drop():
    """For a drop with surface R_s(theta) = R + sum_l a_l P_l(cos theta) and
    a tanh profile symmetric about the surface, the integral of the liquid
    fraction along a ray from the centre is R_s(theta) (exponentially small
    tails); midpoint sampling of the bilinear interpolant keeps it within
    0.05 lattice units."""
    nz, nr, R = 128, 64, 24.0
    coeffs = {2: 1.0, 3: -0.6, 4: 0.4}
    rho_l, rho_g = 2.0, 0.1
    rho = drop_density(nz, nr, nz / 2.0, R, rho_l, rho_g, 1.5, coeffs)
    th = [(m + 0.5) * np.pi / 8 for m in range(8)]
    W = D.interface_radius_weights(nz, nr, nz / 2.0, th)
    got = D.interface_radius(rho, W, rho_l, rho_g)
    want = [R + sum(a * legendre(l, np.cos(t)) for l, a in coeffs.items()) for t in th]
    assert np.max(np.abs(got - np.array(want))) < 0.05


def test_bulk_pressures_balance_across_flat_interface():
    """Mechanical equilibrium of a flat interface (Sec. II.B, pressure of
    the Shan–Chen fluid): once the interface is steady the bulk pressures on
    the two sides agree, while the two densities differ by a factor of 20.
    (At tau = 1 the approach is slow: 3e-3 apart after 10^4 steps, 3e-8
    after 4 x 10^4.)"""
    G = -5.5
    rg, rl = coexistence_densities(G)
    nr = 64
    p = O.make_params(1, nr, G=G, tau=1.0, wall=1, axisym=0)
    _, r = node_coords(1, nr)
    rho = tanh_profile(r, nr / 2.0, rl, rg, 2.0)
    f = O.run(p, O.equilibrium(p, rho, 0 * rho, 0 * rho), 40000)
    rr, _, _ = O.moments(p, f)
    p_l = D.pressure(rr[0:1, :], G)[0, 0]
    p_g = D.pressure(rr[-1:, :], G)[0, 0]
    assert rr[0, 0] / rr[-1, 0] > 20
    assert abs(p_l - p_g) < 1e-6 * abs(p_l)


def _blocks(nz, nr, blocks, rho_l=2.0, rho_g=0.2):
    """Sharp liquid blocks: rows 0..m-1 liquid on columns a .. a+L-1 (mod nz)."""
    rho = np.full((nr, nz), rho_g)
    for a, L, m in blocks:
        for k in range(L):
            rho[:m, (a + k) % nz] = rho_l
    return rho


def test_drops_of_sharp_blocks_are_exact():
    """A block of m liquid rows over L columns with a sharp step and rho_mid
    halfway: the interface crossing is exactly r = m (the last liquid node
    sits at m - 1/2 and rho falls by twice rho_l - rho_mid over one
    spacing), so the volume is pi m^2 L and the centre the block's middle
    column.  One block wraps across the periodic end."""
    nz, nr = 40, 16
    blocks = [(4, 5, 4), (14, 7, 2), (37, 6, 6)]  # the last covers 37..39, 0..2
    rho = _blocks(nz, nr, blocks)
    n, vols, cents = D.drops(rho, 1.1)
    assert n == 3
    # listed from the first gas column (3) onward
    want = [(np.pi * 16 * 5, 6.0), (np.pi * 4 * 7, 17.0), (np.pi * 36 * 6, 39.5)]
    for (v, c), (wv, wc) in zip(zip(vols, cents), want):
        assert v == pytest.approx(wv, rel=1e-14)
        assert c == pytest.approx(wc, abs=1e-12)


def test_drops_of_spheres_and_degenerate_cases():
    """Diffuse spheres of radius a on the axis have volume (4/3) pi a^3 to
    within the midpoint sum over columns (2 %); an unbroken cylinder gives
    n = -1 and pure gas n = 0."""
    nz, nr, rl, rg = 200, 40, 2.0, 0.1
    r = np.arange(nr)[:, None] + 0.5
    z = np.arange(nz)[None, :]
    rho = np.full((nr, nz), rg)
    for zc, a in ((50.0, 12.0), (150.0, 8.0)):
        d = np.sqrt(r * r + (z - zc) ** 2)
        rho = np.maximum(rho, rg + 0.5 * (rl - rg) * (1.0 - np.tanh((d - a) / 1.5)))
    n, vols, cents = D.drops(rho, 0.5 * (rl + rg))
    assert n == 2
    for v, c, (zc, a) in zip(vols, cents, ((50.0, 12.0), (150.0, 8.0))):
        assert v == pytest.approx(4.0 / 3.0 * np.pi * a ** 3, rel=0.02)
        assert c == pytest.approx(zc, abs=0.05)
    cyl = np.where(r < 10.0, rl, rg) * np.ones((1, nz))
    assert D.drops(cyl, 0.5 * (rl + rg))[0] == -1
    assert D.drops(np.full((nr, nz), rg), 0.5 * (rl + rg))[0] == 0
