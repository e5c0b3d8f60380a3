"""The coexistence table the input recipes start drops and threads from
(lbm_inputs/coexistence_tau.json) is what the oracle's flat interface gives:
two entries recomputed here with the script that wrote the table; and the
interpolation reproduces the grid points and stays between them."""
import importlib.util
import os

import pytest

from lbm_inputs import coexistence_densities, scheme_coexistence

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _maker():
    spec = importlib.util.spec_from_file_location("make_coexistence_table",
                                                  os.path.join(ROOT, "tests", "golden", "make_coexistence_table.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


@pytest.mark.parametrize("G,tau", [(-5.5, 0.8), (-5.0, 1.0)])
def test_table_entries_match_the_oracle(G, tau):
    g, l = _maker().flat_interface(G, tau)
    tg, tl = scheme_coexistence(G, tau)
    assert tg == pytest.approx(g, rel=1e-12)
    assert tl == pytest.approx(l, rel=1e-12)


def test_interpolation_and_tau_dependence():
    # at tau = 1 the scheme settles close to the mechanical-stability rule
    g1, l1 = scheme_coexistence(-5.5, 1.0)
    rg, rl = coexistence_densities(-5.5)
    assert l1 == pytest.approx(rl, rel=1e-3) and g1 == pytest.approx(rg, rel=2e-2)
    # at tau = 0.8 the vapour is about 30 % thinner
    g8, l8 = scheme_coexistence(-5.5, 0.8)
    assert 0.6 < g8 / g1 < 0.8 and 0.97 < l8 / l1 < 1.0
    # between grid points the values lie between the neighbours
    gm, lm = scheme_coexistence(-5.55, 0.875)
    lo, hi = scheme_coexistence(-5.5, 0.85), scheme_coexistence(-5.6, 0.9)
    assert min(lo[1], hi[1]) <= lm <= max(lo[1], hi[1])
    with pytest.raises(ValueError):
        scheme_coexistence(-6.0, 0.6)   # the interface diverges there
    with pytest.raises(ValueError):
        scheme_coexistence(-4.0, 1.0)   # outside the table
