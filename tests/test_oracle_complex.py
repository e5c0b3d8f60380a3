"""Pins of the oracle's complex build (complex-step derivatives of the step),
which the adjoint tests use as their reference Jacobian-vector products.

The complex build must be the analytic continuation of the real one: its
real part reproduces the real step bit for bit, and Im(step(f + i h v)) / h
agrees with central finite differences of the real step (Squire and Trapp's
complex-step derivative), as do the derivatives in G and tau."""
import numpy as np
import pytest

import oracle as O
from lbm_inputs import coexistence_densities, drop_density

H = 1e-20


def _state(nz, nr, G, seed):
    rg, rl = coexistence_densities(G)
    rho = drop_density(nz, nr, nz / 2.0, 0.3 * nr, rl, rg, 2.0, {2: 0.5})
    rng = np.random.Generator(np.random.PCG64(seed))
    p = O.make_params(nz, nr, G=G, tau=0.9)
    f = O.equilibrium(p, rho, 0 * rho, 0 * rho) * (1.0 + 0.005 * rng.uniform(-1, 1, size=(9, nr, nz)))
    return f, rng


@pytest.mark.parametrize("wall,axisym", [(0, 1), (1, 1), (1, 0)])
def test_complex_step_matches_real_step_and_fd(wall, axisym):
    nz, nr, G, tau, steps = 24, 12, -5.5, 0.9, 3
    f, rng = _state(nz, nr, G, 5 + wall + 2 * axisym)
    v = rng.standard_normal(f.shape)
    p = O.make_params(nz, nr, G=G, tau=tau, wall=wall, axisym=axisym)
    real = O.run(p, f, steps)
    cplx = O.run(p, f + 1j * H * v, steps, complex_step=True)
    assert np.array_equal(cplx.real, real)
    jv = cplx.imag / H
    h = 1e-6
    fd = (O.run(p, f + h * v, steps) - O.run(p, f - h * v, steps)) / (2 * h)
    assert np.max(np.abs(jv - fd)) < 1e-7 * np.max(np.abs(jv))
    for name in ("G", "tau"):
        kw = {"G_im": H} if name == "G" else {"tau_im": H}
        pc = O.make_params(nz, nr, G=G, tau=tau, wall=wall, axisym=axisym, **kw)
        d = O.run(pc, f.astype(complex), steps, complex_step=True).imag / H
        hp = dict(G=G, tau=tau)
        hm = dict(G=G, tau=tau)
        hp[name] += h
        hm[name] -= h
        fdp = O.run(O.make_params(nz, nr, wall=wall, axisym=axisym, **hp), f, steps)
        fdm = O.run(O.make_params(nz, nr, wall=wall, axisym=axisym, **hm), f, steps)
        fdd = (fdp - fdm) / (2 * h)
        assert np.max(np.abs(d - fdd)) < 1e-6 * np.max(np.abs(d)), name
