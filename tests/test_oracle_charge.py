"""Pins of the oracle's full space charge (Eq. Poisson with holes and dopant
ionization, Sec. II.A.1 and II.A.3) and of the Ohmic-contact potentials
(Sec. II.A.4), against textbook identities that the formulas must obey rather
than against the formulas themselves."""
import numpy as np
import pytest

import synth
from oracle import physics as ph
from oracle import solver

CM3 = 1e-21   # cm^-3 -> nm^-3


def mb(T, **kw):
    return ph.Statistics("mb", T, 1.08, 0.56, holes=True, **kw)


def test_hole_dos_mass_adds_the_two_valence_bands():
    # Eq. EffectiveMass makes N_V of the combined band the sum of the heavy-
    # and light-hole N_V (the DOS scales as m^(3/2))
    T = 300.0
    assert ph.effective_dos(T, ph.SI_M_H) == pytest.approx(
        ph.effective_dos(T, ph.SI_M_HH) + ph.effective_dos(T, ph.SI_M_LH), rel=1e-13)


def test_boltzmann_is_the_nondegenerate_limit_of_fermi_dirac():
    fd = ph.Statistics("fd", 300.0, 1.08, 0.56, holes=True)
    st = mb(300.0)
    kT = ph.kT_eV(300.0)
    for x in (-20.0, -30.0, -45.0):
        phi_n = 0.56 + x * kT                # electrons at E_F - E_C = x kT
        phi_p = 0.56 - 1.12 - x * kT         # holes at E_V - E_F = x kT
        assert fd.density(phi_n) / st.density(phi_n) == pytest.approx(1.0, abs=1e-8)
        assert fd.hole_density(phi_p) / st.hole_density(phi_p) == pytest.approx(1.0, abs=1e-8)


def test_mass_action_law():
    # n p = N_C N_V exp(-Eg/kT) at any potential (Boltzmann statistics)
    st = mb(300.0)
    ni2 = st.Nc * st.Nv * np.exp(-st.Eg / st.kT)
    for phi in (-0.4, -0.1, 0.0, 0.2, 0.5):
        assert st.density(phi) * st.hole_density(phi) == pytest.approx(ni2, rel=1e-12)


def test_intrinsic_level():
    # n = p without dopants at phi = Ec0 - Eg/2 + (kT/2) ln(N_V/N_C)
    st = mb(300.0)
    expect = st.Ec0 - st.Eg / 2 + 0.5 * st.kT * np.log(st.Nv / st.Nc)
    assert ph.neutral_root(st, 0.0) == pytest.approx(expect, abs=1e-12)


@pytest.mark.parametrize("T", [30.0, 77.0, 300.0])
def test_dopant_ionization_obeys_the_saha_relation(T):
    # detailed balance between the band and the impurity level (Boltzmann):
    # n N_D+ / (N_D - N_D+) = (N_C / g_D) exp(-E_d/kT), same for acceptors
    # (evaluated within a few kT of each level, where both charge states exist)
    st = mb(T, ionization="incomplete")
    nd, na = 1e17 * CM3, 3e16 * CM3
    for s in (-3.0, 0.0, 2.0):
        phi_d = st.Ec0 - st.Ed + s * st.kT             # E_F - E_D = s kT
        phi_a = st.Ec0 - st.Eg + st.Ea - s * st.kT     # E_A - E_F = s kT
        dplus, _ = st.ionized(phi_d, nd, na)
        _, aminus = st.ionized(phi_a, nd, na)
        lhs_d = st.density(phi_d) * dplus / (nd - dplus)
        lhs_a = st.hole_density(phi_a) * aminus / (na - aminus)
        assert lhs_d == pytest.approx(st.Nc / st.gD * np.exp(-st.Ed / st.kT), rel=1e-9)
        assert lhs_a == pytest.approx(st.Nv / st.gA * np.exp(-st.Ea / st.kT), rel=1e-9)


@pytest.mark.parametrize("stat,T", [("mb", 77.0), ("fd", 4.0), ("fd", 300.0)])
def test_space_charge_derivative_matches_differences(stat, T):
    st = ph.Statistics(stat, T, 1.08, 0.56, holes=True, ionization="incomplete")
    nd, na = 2e18 * CM3, 1e15 * CM3
    kT = ph.kT_eV(T)
    for phi in np.linspace(-0.7, 0.7, 15):
        h = 1e-4 * kT
        num = (st.rho(phi + h, nd - na, nd, na) - st.rho(phi - h, nd - na, nd, na)) / (2 * h)
        ana = st.drho(phi, nd, na)
        assert ana <= 0.0
        assert ana == pytest.approx(num, rel=1e-5, abs=1e-12 * abs(st.rho(phi, nd - na, nd, na)) / kT + 1e-300)


@pytest.mark.parametrize("T", [77.0, 300.0])
def test_ohmic_potential_boltzmann_complete_ionization(T):
    st = mb(T)
    nd, na = 1e18 * CM3, 1e16 * CM3
    phn = ph.ohmic_potential(st, nd, 0.0)
    php = ph.ohmic_potential(st, 0.0, na)
    assert st.density(phn) == pytest.approx(nd, rel=1e-12)       # majority carriers balance the dopants
    assert st.hole_density(php) == pytest.approx(na, rel=1e-12)
    # the built-in potential of the junction the two contacts bound:
    # kT ln(N_A N_D / n_i^2) with n_i^2 from the mass-action law
    ni2 = st.Nc * st.Nv * np.exp(-st.Eg / st.kT)
    assert phn - php == pytest.approx(st.kT * np.log(nd * na / ni2), rel=1e-12)
    # applied voltage shifts the contact rigidly
    assert ph.ohmic_potential(st, nd, 0.0, Va=0.3) == pytest.approx(phn + 0.3, abs=1e-15)


@pytest.mark.parametrize("T", [30.0, 77.0, 300.0])
def test_ohmic_potential_incomplete_ionization_is_neutral(T):
    # majority carriers balance the ionized dopants at the contact
    st = mb(T, ionization="incomplete")
    nd, na = 1e17 * CM3, 1e17 * CM3
    phn = ph.ohmic_potential(st, nd, 0.0)
    php = ph.ohmic_potential(st, 0.0, na)
    dplus, _ = st.ionized(phn, nd, 0.0)
    _, aminus = st.ionized(php, 0.0, na)
    assert st.density(phn) == pytest.approx(dplus, rel=1e-10)
    assert st.hole_density(php) == pytest.approx(aminus, rel=1e-10)   # fixes the sign of E_a
    # and it is the neutral point of the full charge (minority carriers and
    # the opposite dopant are negligible here)
    assert ph.neutral_root(st, 0.0, nd, 0.0) == pytest.approx(phn, abs=1e-9)
    assert ph.neutral_root(st, 0.0, 0.0, na) == pytest.approx(php, abs=1e-9)


def test_ohmic_low_temperature_log_form():
    # where both are representable the low-T form of ln y matches the exact
    # one to the size of the dropped terms; at 4 K only the low-T form exists
    # and the contact is still neutral
    nd = 1e17 * CM3
    st = mb(20.0, ionization="incomplete")
    exact = ph.ohmic_potential(st, nd, 0.0)
    approx = ph.ohmic_potential(st, nd, 0.0, low_T_log_min=1.0)
    assert approx == pytest.approx(exact, abs=1e-6)
    cold = mb(4.0, ionization="incomplete")
    phn = ph.ohmic_potential(cold, nd, 0.0)
    dplus, _ = cold.ionized(phn, nd, 0.0)
    assert cold.density(phn) == pytest.approx(dplus, rel=1e-9)


def test_ohmic_potential_fermi_dirac_within_the_inverse_error():
    st = ph.Statistics("fd", 300.0, 1.08, 0.56, holes=True)
    for nd in (1e15 * CM3, 1e19 * CM3, 1e20 * CM3):
        phn = ph.ohmic_potential(st, nd, 0.0)
        assert st.density(phn) == pytest.approx(nd, rel=0.03)     # Eq. FDintInverse, < 0.6 % in eta


def ohmic_block(stat, T, ionization, nd, na, n=(5, 5, 9)):
    dev = synth.doped_block("blk", *n, (20.0, 20.0, 40.0), lambda x, y, z: nd, lambda x, y, z: na,
                            [("bottom", "bottom")], stat=stat, T_K=T, holes=True, ionization=ionization)
    return dev


@pytest.mark.parametrize("ionization", ["complete", "incomplete"])
def test_uniform_block_with_ohmic_contact_stays_neutral(ionization):
    # a uniformly doped block held at its neutral potential on one face and
    # flux-free elsewhere has no field: phi is the neutral root everywhere
    st = mb(77.0, ionization=ionization)
    nd, na = 5e17 * CM3, 1e15 * CM3
    root = ph.neutral_root(st, nd - na, nd, na)
    dev = ohmic_block("mb", 77.0, ionization, nd, na)
    dev.dir_val[:] = root
    prob, res = solver.solve(dev, atol=1e-12)
    assert res.status == "ok"
    assert np.abs(res.phi - root).max() < 1e-12
    # the paper's closed form (majority carriers only) sits on the neutral
    # point (with incomplete ionization it takes the majority dopant alone:
    # compared on an uncompensated contact)
    if ionization == "complete":
        assert abs(ph.ohmic_potential(st, nd, na) - root) < 1e-9
    else:
        assert abs(ph.ohmic_potential(st, nd, 0.0) - ph.neutral_root(st, nd, nd, 0.0)) < 1e-9


def test_pn_junction_between_ohmic_contacts():
    # abrupt p-n junction (p below z = 100 nm, n above), Boltzmann statistics,
    # complete ionization: far from the junction the potential is flat at the
    # contacts' values, across it the drop is the built-in potential and the
    # net space charge integrates to (almost) zero
    T = 300.0
    st = mb(T)
    nd, na = 1e18 * CM3, 1e18 * CM3
    dev = synth.doped_block("pn", 3, 3, 201, (10.0, 10.0, 200.0),
                            lambda x, y, z: np.where(z > 100.0, nd, 0.0),
                            lambda x, y, z: np.where(z > 100.0, 0.0, na),
                            [("p", "bottom"), ("n", "top")], stat="mb", T_K=T, holes=True)
    php, phn = ph.ohmic_potential(st, 0.0, na), ph.ohmic_potential(st, nd, 0.0)
    dev.dir_val[:] = [php, phn]
    prob, res = solver.solve(dev, atol=1e-10)
    assert res.status == "ok"
    z = dev.z
    col = res.phi.reshape(dev.nz, dev.ny, dev.nx)[:, 1, 1]
    assert np.all(np.diff(col) >= -1e-12)                       # monotone
    assert abs(col[np.argmin(np.abs(z - 10.0))] - php) < 1e-3   # flat, neutral p side
    assert abs(col[np.argmin(np.abs(z - 190.0))] - phn) < 1e-3  # flat, neutral n side
    vbi = st.kT * np.log(nd * na / (st.Nc * st.Nv * np.exp(-st.Eg / st.kT)))
    assert phn - php == pytest.approx(vbi, rel=1e-12)
    # depletion width from the depletion approximation, 2 sqrt(eps Vbi / (q N)) for N_A = N_D
    half = np.sqrt(11.7 * vbi / (ph.KAPPA * nd))
    mid = 0.5 * (php + phn)
    inside = np.abs(col - mid) < 0.45 * vbi
    w = z[inside].max() - z[inside].min()
    assert 0.5 * 2 * half < w < 2 * half
