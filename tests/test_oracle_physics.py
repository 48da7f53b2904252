"""Pins of the reference carrier statistics against quantities the paper and
the mathematics fix (quadrature of the defining integral, asymptotes, the
printed error bounds, textbook constants, closed-form inverses)."""
import json
import os

import numpy as np
import pytest

from oracle import physics as ph


@pytest.fixture(scope="module")
def paper(golden_dir):
    with open(os.path.join(golden_dir, "paper_values.json")) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def consts(golden_dir):
    with open(os.path.join(golden_dir, "constants.json")) as f:
        return json.load(f)


def test_fd_half_within_printed_bound(paper):
    # Eq. FDIntApprox vs Eq. FDIntegral evaluated by quadrature.
    x = np.linspace(-60.0, 100.0, 641)
    exact = ph.fd_half_quadrature(x)
    rel = np.abs(ph.fd_half(x) / exact - 1.0)
    assert rel.max() < paper["fd_half_max_rel_err"]["value"]
    # the bound is nearly attained (Bednarczyk form, not an exact integral):
    assert rel.max() > 0.003
    assert abs(x[rel.argmax()] - 3.5) < 0.5


def test_fd_half_asymptotes():
    # x -> -inf: exp(x); x -> +inf: 4 x^1.5 / (3 sqrt(pi))  (Fig. FDIntCmprsn)
    for x in (-45.0, -49.9):
        assert ph.fd_half(np.array([x]))[0] / np.exp(x) == pytest.approx(1.0, abs=1e-15)
    for x in (1e4, 1e6):
        deg = 4.0 * x ** 1.5 / (3.0 * np.sqrt(np.pi))
        assert ph.fd_half(np.array([x]))[0] / deg == pytest.approx(1.0, rel=50.0 / x ** 3 + 1e-15)


def test_switch_continuity(paper):
    s = paper["fd_switch_x"]["value"]
    lo = ph.fd_half(np.array([np.nextafter(s, -np.inf)]))[0]
    hi = ph.fd_half(np.array([s]))[0]
    assert abs(hi / lo - 1.0) < 1e-14
    dlo = ph.fd_half_prime(np.array([np.nextafter(s, -np.inf)]))[0]
    dhi = ph.fd_half_prime(np.array([s]))[0]
    assert abs(dhi / dlo - 1.0) < 1e-12


def test_fd_derivative_matches_central_difference():
    x = np.concatenate([np.linspace(-49.0, 60.0, 437), [-60.0, -55.0, 200.0, 551.0]])
    h = np.where(np.abs(x) > 100, 1e-3, 1e-5)
    fd = (ph.fd_half(x + h) - ph.fd_half(x - h)) / (2 * h)
    an = ph.fd_half_prime(x)
    assert np.max(np.abs(an / fd - 1.0)) < 1e-8
    assert np.all(an > 0)           # n nondecreasing -> convex energy, unique solution


def test_constants_match_independent_values(consts):
    assert ph.KAPPA == pytest.approx(consts["kappa_V_nm"]["value"], rel=1e-14)
    assert ph.thomas_fermi_coeff(1.08) == pytest.approx(consts["C_TF_m1.08"]["value"], rel=1e-9)
    assert ph.effective_dos(4.0, 1.08) == pytest.approx(consts["N_C_4K_m1.08"]["value"], rel=1e-6)
    assert ph.kT_eV(4.0) == pytest.approx(consts["kT_4K_eV"]["value"], rel=1e-6)
    tb = consts["N_C_300K_Si_textbook"]
    assert ph.effective_dos(300.0, 1.08) == pytest.approx(tb["value"], rel=tb["rtol"])
    md = consts["m_dos_Si"]
    assert ph.dos_mass(0.98, 0.19) == pytest.approx(md["value"], rel=md["rtol"])


def test_tf_is_degenerate_fd_limit():
    # Appendix A: n = N_C F_1/2(eta); for eta >> 1 F_1/2 -> 4 eta^1.5/(3 sqrt(pi)),
    # which must reproduce the T = 0 density C_TF u^1.5 for any T (N_C ~ T^1.5).
    for T in (0.5, 4.0, 50.0):
        fd = ph.Statistics("fd", T, 1.08, 0.0)
        tf = ph.Statistics("tf", 0.0, 1.08, 0.0)
        u = np.array([0.05, 0.19, 0.6])
        eta = u / fd.kT
        ratio = fd.density(u) / tf.density(u)
        # Bednarczyk's large-x correction is 12.6/x^3 relative
        assert np.allclose(ratio, 1.0, rtol=20.0 / eta.min() ** 3 + 1e-13, atol=0)


def test_tf_neutral_point_closed_form():
    # free-electron Fermi energy: E_F - E_C = hbar^2 (3 pi^2 n)^(2/3) / (2 m*)
    st = ph.Statistics("tf", 0.0, 1.08, 0.56)
    for nd in (1e-4, 1e-3, 3e-2):
        ef = ph.HBAR ** 2 * (3 * np.pi ** 2 * nd * 1e27) ** (2.0 / 3.0) / (2 * 1.08 * ph.M0) / ph.Q_E
        assert st.neutral_potential(nd) == pytest.approx(0.56 + ef, rel=1e-13)


def test_fd_neutral_point_vs_nilsson(paper):
    # Eq. FDintInverse recovers the degeneracy of a neutral donor-doped bulk
    # within its stated error (measured on the density it implies).
    st = ph.Statistics("fd", 4.0, 1.08, 0.56)
    for nd in (1e-7, 1e-5, 1e-4, 1e-3, 1e-2):
        phin = st.neutral_potential(nd)
        eta_nils = ph.nilsson_inverse(np.array([nd / st.Nc]))[0]
        n_nils = st.Nc * ph.fd_half_quadrature(np.array([eta_nils]))[0]
        n_exact = st.Nc * ph.fd_half_quadrature(np.array([(phin - 0.56) / st.kT]))[0]
        # n_exact differs from nd only by the Bednarczyk error (< 0.4%)
        assert abs(n_nils / n_exact - 1.0) < paper["nilsson_max_err"]["value"] + paper["fd_half_max_rel_err"]["value"]
        assert abs(n_exact / nd - 1.0) < paper["fd_half_max_rel_err"]["value"]


def test_nilsson_inverse_bound(paper):
    x = np.linspace(-20.0, 60.0, 161)
    u = ph.fd_half_quadrature(x)
    eta = ph.nilsson_inverse(u)
    rel_u = np.abs(ph.fd_half_quadrature(eta) / u - 1.0)
    assert rel_u.max() < paper["nilsson_max_err"]["value"]


def test_statistics_edge_cases():
    tf = ph.Statistics("tf", 0.0, 1.08, 0.56)
    assert tf.density(np.array([0.56, 0.0, -3.0])).tolist() == [0.0, 0.0, 0.0]
    assert tf.ddensity(np.array([0.56])).tolist() == [0.0]
    fd = ph.Statistics("fd", 4.0, 1.08, 0.56)
    # deep depletion underflows to an exact zero (eta ~ -1625)
    assert fd.density(np.array([0.0]))[0] == 0.0
    with pytest.raises(ValueError):
        ph.Statistics("fd", 0.0)
    lin = ph.Statistics("linear")
    assert not np.any(lin.density(np.linspace(-1, 3, 9)))
