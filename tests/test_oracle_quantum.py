"""Pins of the oracle's predictor-corrector electron density (Eqs. pcPoisson,
ApproxEDens3DConfined, ApproxEDens1DConfined): occupation limits counted over
a whole block, the first-order perturbation property that fixes the sign of
the potential term, the 2D density of states in the degenerate limit of the
1D form, and the Newton system's Jacobian and uniqueness."""
import numpy as np
import pytest

import synth
from oracle import physics as ph
from oracle import solver
from oracle.quantum import QuantumDensity


def uniform_block(n_states, E, T=4.0, phi_k=0.3, conf=3):
    dev = synth.doped_block("qb", 5, 4, 6, (10.0, 8.0, 12.0), lambda x, y, z: 0.0, lambda x, y, z: 0.0,
                            [], stat="fd", T_K=T, holes=False)
    V = 10.0 * 8.0 * 12.0
    psi2 = np.full((n_states, dev.n_nodes), 1.0 / V)
    st = synth.QuantumStates(psi2=psi2, phi_k=np.full(dev.n_nodes, phi_k), E_i=np.asarray(E, float),
                             confinement=conf)
    return synth.with_quantum(dev, st)


def test_deep_levels_hold_four_electrons_each():
    # a normalised state far below E_F is fully occupied: 2 spins x 2 valleys
    dev = uniform_block(3, [-1.0, -0.8, -0.9])
    po = solver.make_problem(dev)
    box = (-1, 11, -1, 9, -1, 13)
    assert po.count(np.full(dev.n_nodes, 0.3), box) == pytest.approx(12.0, rel=1e-12)
    # and a level at E_F (phi = phi_k) is half occupied; far above, empty
    dev = uniform_block(2, [0.0, 1.0])
    po = solver.make_problem(dev)
    assert po.count(np.full(dev.n_nodes, 0.3), box) == pytest.approx(2.0, rel=1e-12)


@pytest.mark.parametrize("conf", [3, 1])
def test_potential_rise_lowers_every_level(conf):
    # first-order perturbation: phi = phi_k + d is the same as levels E_i - d
    # at phi_k (a potential rise lowers the electron energy); the opposite
    # sign of the potential term would fail this
    rng = np.random.default_rng(1)
    N = 50
    psi2 = rng.uniform(0.0, 1e-3, (3, N))
    phik = rng.uniform(-0.1, 0.4, N)
    E = np.array([-0.003, 0.001, 0.004])
    d = 0.0017
    a = QuantumDensity(psi2, phik, E, 4.0, conf).at_nodes(phik + d)[0]
    b = QuantumDensity(psi2, phik, E - d, 4.0, conf).at_nodes(phik)[0]
    assert np.allclose(a, b, rtol=1e-13, atol=0)
    n, dn = QuantumDensity(psi2, phik, E, 4.0, conf).at_nodes(phik + rng.normal(0, 0.002, N))
    assert np.all(dn >= 0)            # n~ grows with phi: the Newton system stays SPD


def test_one_dimensional_form_degenerate_limit_is_the_2d_density_of_states():
    # deep in the degenerate limit ln(1 + e^x) -> x, so n~ -> g2D (E_F - E_i) |psi|^2
    # with g2D = g_s g_v m_t / (2 pi hbar^2), g_s = g_v = 2, independent of T
    m_t = 0.19
    g2d = 2 * 2 * m_t * 9.1093837015e-31 / (2 * np.pi * (1.054571817e-34) ** 2) * 1.602176634e-19 * 1e-18
    psi2 = np.array([[0.05]])          # nm^-1
    for T in (1.0, 2.0):
        q = QuantumDensity(psi2, np.zeros(1), [-0.02], T, confinement=1, m_t=m_t)
        n = q.at_nodes(np.zeros(1))[0][0]
        assert n == pytest.approx(g2d * 0.02 * 0.05, rel=1e-12)
    # and in the nondegenerate limit a Boltzmann tail: P |psi|^2 e^x
    T = 300.0
    q = QuantumDensity(psi2, np.zeros(1), [0.5], T, confinement=1, m_t=m_t)
    kT = ph.kT_eV(T)
    assert q.at_nodes(np.zeros(1))[0][0] == pytest.approx(q.P * 0.05 * np.exp(-0.5 / kT), rel=1e-12)
    assert q.P == pytest.approx(g2d * kT, rel=1e-12)


def pc_stack():
    volts = np.array([2.0, 1.8, 0.9, 1.1, 0.7])
    dev = synth.double_dot_device("pc", 15, 13, 11, volts)
    _, res = solver.solve(dev, atol=1e-10)
    st = synth.box_states(dev, (10.0, 60.0, 80.0, 120.0, 75.0, 90.0), 4, res.phi, seed=3)
    return synth.with_quantum(dev, st), res.phi


def test_pc_jacobian_matches_differences_and_is_symmetric():
    dev, phi0 = pc_stack()
    po, res = solver.solve(dev, atol=1e-10)
    assert res.status == "ok"
    rng = np.random.default_rng(4)
    phi = po.with_dirichlet(res.phi + 0.005 * rng.standard_normal(po.mesh.N))
    v = np.where(po.free, rng.standard_normal(po.mesh.N), 0.0)
    h = 1e-7
    fd = (po.residual(phi + h * v) - po.residual(phi - h * v)) / (2 * h)
    jv = po.jv(phi, v)
    f = po.free
    assert np.abs(jv[f] - fd[f]).max() < 1e-6 * np.abs(jv[f]).max()
    J = po.jacobian_free(phi)
    assert abs(J - J.T).max() < 1e-12 * abs(J).max()


def test_pc_solution_unique_and_counts_states():
    dev, phi0 = pc_stack()
    po = solver.make_problem(dev)
    a = solver.newton(po, atol=1e-11)
    b = solver.newton(po, phi0=po.with_dirichlet(phi0 + 0.05), atol=1e-11)
    assert a.status == b.status == "ok"
    assert np.abs(a.phi - b.phi).max() < 1e-9
    # the dot holds at most 4 electrons per state (here about 1 level is
    # occupied), and none outside the states' box
    n = po.count(a.phi, (0, 200, 0, 200, 0, 100))
    assert 0.5 < n < 16.0
    assert po.count(a.phi, (100, 200, 0, 200, 0, 100)) == 0.0


def test_quantum_region_selects_the_electron_model():
    # outside the region the statistics hold: an empty region reproduces the
    # semiclassical residual, a full one the states-only residual
    dev, phi0 = pc_stack()
    E = dev.n_elems
    rng = np.random.default_rng(9)
    phi = phi0 + 0.01 * rng.standard_normal(dev.n_nodes)
    semi = solver.make_problem(synth.Device(**{**dev.__dict__, "quantum": None}))
    q_all = solver.make_problem(dev)
    st = dev.quantum
    none_reg = synth.QuantumStates(st.psi2, st.phi_k, st.E_i, region=np.zeros(E, bool))
    full_reg = synth.QuantumStates(st.psi2, st.phi_k, st.E_i, region=np.ones(E, bool))
    assert np.array_equal(solver.make_problem(synth.with_quantum(dev, none_reg)).residual(phi), semi.residual(phi))
    assert np.array_equal(solver.make_problem(synth.with_quantum(dev, full_reg)).residual(phi), q_all.residual(phi))
