"""Pins of the oracle's boundary rules (Sec. II.E) and conservation
properties: rest-state invariance, the streaming links at the axis and the
wall, exact 2D mass and momentum conservation, the reduction of the
axisymmetric scheme to the planar one for r-independent states, and the
paper's remark on 3D versus 2D mass."""
import numpy as np
import pytest

import oracle as O
from lbm_inputs import coexistence_densities, drop_density
import oracle.diagnostics as D


@pytest.mark.parametrize("wall", [0, 1])
@pytest.mark.parametrize("G,rho_val", [(0.0, 0.83), (-5.5, 0.1), (-5.5, 2.3)])
def test_rest_state_is_invariant(wall, G, rho_val):
    """Uniform density at rest: the Shan–Chen force, the derivative terms and
    the axisymmetric sources all vanish, and every boundary link returns a
    population of the same weight, so f stays W_i rho (to round-off) for 1000
    steps.  A wrong ghost rule for psi (e.g. zero ghosts at the wall) makes
    the force non-zero on the boundary rows at the first step.  With G != 0
    the density is taken outside the spinodal region (dp/drho > 0 for the
    equation of state of Sec. II.A), where a uniform state is stable."""
    nz, nr = 10, 8
    rho = np.full((nr, nz), rho_val)
    p = O.make_params(nz, nr, G=G, tau=0.9, wall=wall, axisym=1)
    f0 = O.equilibrium(p, rho, 0 * rho, 0 * rho)
    f1 = O.run(p, f0, 1000)
    assert np.abs(f1 - f0).max() < 1e-13


def _labelled(nz, nr):
    return np.arange(9 * nz * nr, dtype=np.float64).reshape(9, nr, nz) + 1.0


@pytest.mark.parametrize("wall", [0, 1])
def test_streaming_is_a_permutation(wall):
    """Every (node, direction) receives exactly one population: the
    mid-grid specular axis, mid-grid bounce-back and mid-grid specular wall
    are all one-to-one link maps."""
    nz, nr = 5, 6
    p = O.make_params(nz, nr, wall=wall)
    f = _labelled(nz, nr)
    out = O.stream(p, f)
    assert sorted(out.ravel().tolist()) == sorted(f.ravel().tolist())


def _val(f, i, r, z):
    return f[i, r, z]


def test_axis_links_are_specular():
    """A population leaving row 0 towards r < 0 re-enters row 0 at the
    mirrored position with its radial velocity reversed (Sec. II.E)."""
    nz, nr = 5, 6
    p = O.make_params(nz, nr, wall=0)
    f = _labelled(nz, nr)
    out = O.stream(p, f)
    z = 2
    assert out[2, 0, z] == f[4, 0, z]             # (0,-1) -> (0,+1), same column
    assert out[6, 0, z - 1] == f[7, 0, z]         # (-1,-1) -> (-1,+1) at z-1
    assert out[5, 0, z + 1] == f[8, 0, z]         # (+1,-1) -> (+1,+1) at z+1
    # periodic seam in z
    assert out[6, 0, nz - 1] == f[7, 0, 0]


def test_noslip_wall_is_bounce_back():
    nz, nr = 5, 6
    p = O.make_params(nz, nr, wall=0)
    f = _labelled(nz, nr)
    out = O.stream(p, f)
    z, top = 3, nr - 1
    assert out[4, top, z] == f[2, top, z]
    assert out[7, top, z] == f[5, top, z]
    assert out[8, top, z] == f[6, top, z]


def test_freeslip_wall_is_specular():
    nz, nr = 5, 6
    p = O.make_params(nz, nr, wall=1)
    f = _labelled(nz, nr)
    out = O.stream(p, f)
    z, top = 3, nr - 1
    assert out[4, top, z] == f[2, top, z]
    assert out[8, top, z + 1] == f[5, top, z]
    assert out[7, top, z - 1] == f[6, top, z]


def test_interior_streaming():
    nz, nr = 5, 6
    p = O.make_params(nz, nr, wall=0)
    f = _labelled(nz, nr)
    out = O.stream(p, f)
    assert out[1, 2, 3] == f[1, 2, 2]
    assert out[5, 3, 3] == f[5, 2, 2]
    assert out[7, 2, 1] == f[7, 3, 2]
    assert out[3, 2, 4] == f[3, 2, 0]  # periodic seam


def _drop(G=-5.5, nz=48, nr=24, tau=1.0, wall=0, axisym=1, R=9.0):
    rg, rl = coexistence_densities(G)
    rho = drop_density(nz, nr, nz / 2.0, R, rl, rg, 2.0, {2: 1.5})
    p = O.make_params(nz, nr, G=G, tau=tau, wall=wall, axisym=axisym)
    return p, O.equilibrium(p, rho, 0 * rho, 0 * rho)


@pytest.mark.parametrize("wall", [0, 1])
def test_planar_mode_conserves_mass_exactly(wall):
    """Without the axisymmetric terms the scheme is the textbook D2Q9
    Shan–Chen model: BGK conserves density locally and every boundary link
    is a permutation, so sum(rho) is conserved to round-off."""
    p, f = _drop(wall=wall, axisym=0)
    m0 = f.sum()
    f = O.run(p, f, 300)
    assert abs(f.sum() - m0) / m0 < 1e-13


def test_planar_freeslip_conserves_axial_momentum():
    """Planar mode with specular walls: the Shan–Chen force is a sum of
    antisymmetric pair terms (including the pairs across the mirror planes)
    and specular reflection keeps c_z, so the total axial momentum
    sum(c_z f) is conserved to round-off, even for a moving drop."""
    G = -5.5
    rg, rl = coexistence_densities(G)
    nz, nr = 48, 24
    rho = drop_density(nz, nr, 24.0, 8.0, rl, rg, 2.0, {2: 1.0})
    uz = 0.01 * np.sin(2 * np.pi * np.arange(nz) / nz)[None, :] * np.ones((nr, 1))
    p = O.make_params(nz, nr, G=G, tau=1.0, wall=1, axisym=0)
    f = O.equilibrium(p, rho, uz, 0 * rho)
    cz, _, _ = O.lattice()
    P0 = (cz[:, None, None] * f).sum()
    f = O.run(p, f, 200)
    P1 = (cz[:, None, None] * f).sum()
    assert abs(P1 - P0) < 1e-12 * f.sum()
    assert abs(P0) < 1e-12  # the initial momentum is zero by symmetry...
    fl = O.fields(p, f)
    assert np.abs(fl["u_z"]).max() > 1e-5  # ...but the drop is moving


def test_r_independent_state_sees_no_axisymmetric_terms():
    """Sec. II.C/II.D: for a planar slab normal to z with a free-slip wall,
    d_r psi = 0, F_r = 0 and u_r = 0, so F^{gamma,sym} and h vanish and the
    axisymmetric scheme evolves exactly like the planar one."""
    G = -5.5
    rg, rl = coexistence_densities(G)
    nz, nr = 64, 8
    z = np.arange(nz, dtype=float)[None, :] * np.ones((nr, 1))
    from lbm_inputs import tanh_profile
    rho = tanh_profile(np.abs(z - 32.0), 12.0, rl, rg, 2.0)
    out = []
    for axisym in (0, 1):
        p = O.make_params(nz, nr, G=G, tau=1.0, wall=1, axisym=axisym)
        out.append(O.run(p, O.equilibrium(p, rho, 0 * rho, 0 * rho), 500))
    assert np.abs(out[0] - out[1]).max() < 1e-12
    p = O.make_params(nz, nr, G=G, tau=1.0, wall=1, axisym=1)
    fl = O.fields(p, out[1])
    assert np.abs(fl["fsym_r"]).max() < 1e-13 and np.abs(fl["h"]).max() < 1e-13
    assert np.abs(fl["u_z"]).max() > 1e-6


def test_three_dimensional_mass_is_the_conserved_one():
    """Sec. II.C, validation note: in the axisymmetric scheme the 2D mass
    changes while the 3D mass (2 pi r weighting) is conserved with good
    accuracy.  For a drop relaxing towards its equilibrium shape the 3D mass
    drifts far less than the 2D mass."""
    p, f = _drop(tau=1.0, wall=1)
    rho0, _, _ = O.moments(p, f)
    f = O.run(p, f, 1000)
    rho1, _, _ = O.moments(p, f)
    d3 = abs(D.mass_3d(rho1) - D.mass_3d(rho0)) / D.mass_3d(rho0)
    d2 = abs(D.mass_2d(rho1) - D.mass_2d(rho0)) / D.mass_2d(rho0)
    assert d3 < 2e-3
    assert d2 > 5.0 * d3
