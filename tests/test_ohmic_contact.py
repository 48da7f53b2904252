"""The library's Ohmic-contact potential (a host computation, Sec. II.A.4)
against the oracle's, and against the neutrality it is defined by, over
statistics, ionization models, dopant densities, temperatures and the
low-temperature form of the logarithm."""
import numpy as np
import pytest

from oracle import physics as ph
from paper_1403_7561_amd import qe

CM3 = 1e-21


def both(stat, T, ionization, **kw):
    o = ph.Statistics(stat, T, 1.08, 0.56, holes=True, ionization=ionization, **kw)
    g = qe.Physics(stat=stat, T_K=T, m_eff=1.08, Ec0_eV=0.56, holes=True, ionization=ionization, **kw)
    return o, g


@pytest.mark.parametrize("stat", ["mb", "fd"])
@pytest.mark.parametrize("ionization", ["complete", "incomplete"])
@pytest.mark.parametrize("T", [4.0, 30.0, 77.0, 300.0])
def test_matches_oracle(stat, ionization, T):
    o, g = both(stat, T, ionization)
    for nd, na in [(1e15, 0.0), (1e18, 1e16), (0.0, 1e15), (3e16, 2e19), (1e20, 0.0)]:
        nd, na = nd * CM3, na * CM3
        for va in (0.0, -0.25):
            want = ph.ohmic_potential(o, nd, na, Va=va)
            got = qe.qe_ohmic_potential(g, nd, na, va)
            assert got == pytest.approx(want, abs=1e-12 + 1e-13 * abs(want)), (nd, na, va)


@pytest.mark.parametrize("gD,gA", [(2.0, 4.0), (3.0, 1.5)])
def test_incomplete_ionization_contact_is_neutral_for_any_degeneracy(gD, gA):
    # the library solves g y^2 + y = K for any degeneracy factor; the
    # majority carriers then balance the ionised majority dopant exactly
    o, g = both("mb", 50.0, "incomplete", gD=gD, gA=gA)
    nd = 2e17 * CM3
    phn = qe.qe_ohmic_potential(g, nd, 0.0)
    php = qe.qe_ohmic_potential(g, 0.0, nd)
    dplus, _ = o.ionized(phn, nd, 0.0)
    _, aminus = o.ionized(php, 0.0, nd)
    assert o.density(phn) == pytest.approx(dplus, rel=1e-11)
    assert o.hole_density(php) == pytest.approx(aminus, rel=1e-11)


def test_low_temperature_branch_is_continuous():
    # around the switch to the leading-order logarithm (4 g K = 1e300) the two
    # forms differ by far less than kT
    o, g = both("mb", 4.0, "incomplete")
    kT = o.kT
    # pick N_D so that ln(8 K) straddles ln(1e300) for the donor level
    lnK_switch = np.log(1e300) - np.log(8.0)
    Nc = o.Nc
    for d in (-1e-3, 1e-3):
        nd = Nc * np.exp(lnK_switch + d - o.Ed / kT)
        phn = qe.qe_ohmic_potential(g, nd, 0.0)
        dplus, _ = o.ionized(phn, nd, 0.0)
        assert o.density(phn) == pytest.approx(dplus, rel=1e-9)
