"""Shared helpers of the GPU parity tests: device set-up and sampled oracle
evaluations for meshes too large to assemble."""
import numpy as np

import synth
from oracle import solver


def oracle_problem(dev):
    return solver.make_problem(dev)


def sub_device(dev, i, j, k):
    """The (up to) 3x3x3-node block of ``dev`` around node (i, j, k) with all
    its elements, every node free.  Returns (sub-device, index of the centre)."""
    i0, i1 = max(i - 1, 0), min(i + 1, dev.nx - 1)
    j0, j1 = max(j - 1, 0), min(j + 1, dev.ny - 1)
    k0, k1 = max(k - 1, 0), min(k + 1, dev.nz - 1)
    ex, ey = dev.nx - 1, dev.ny - 1
    ei = np.arange(i0, i1)
    ej = np.arange(j0, j1)
    ek = np.arange(k0, k1)
    K, J, I = np.meshgrid(ek, ej, ei, indexing="ij")
    el = (I + ex * (J + ey * K)).ravel()
    snx, sny, snz = i1 - i0 + 1, j1 - j0 + 1, k1 - k0 + 1
    sub = synth.Device(name="sub", x=dev.x[i0:i1 + 1], y=dev.y[j0:j1 + 1], z=dev.z[k0:k1 + 1],
                       eps_r=dev.eps_r[el], semi=dev.semi[el], net_doping=dev.net_doping[el],
                       dir_id=np.full(snx * sny * snz, -1, np.int32), dir_val=np.zeros(0),
                       stat=dev.stat, T_K=dev.T_K, m_eff=dev.m_eff, Ec0_eV=dev.Ec0_eV,
                       holes=dev.holes, ionization=dev.ionization,
                       donors=None if dev.donors is None else dev.donors[el],
                       acceptors=None if dev.acceptors is None else dev.acceptors[el])
    kk, jj, ii = np.meshgrid(np.arange(k0, k1 + 1), np.arange(j0, j1 + 1), np.arange(i0, i1 + 1),
                             indexing="ij")
    glob = (ii + dev.nx * (jj + dev.ny * kk)).ravel()
    centre = (i - i0) + snx * ((j - j0) + sny * (k - k0))
    return sub, glob, centre


def sampled_residual(dev, phi, nodes):
    """Oracle residual F_n (zero on Dirichlet nodes) at the given node indices,
    each from its own small sub-mesh (F_n only depends on the 8 elements around n)."""
    out = np.empty(len(nodes))
    for t, n in enumerate(nodes):
        n = int(n)
        i, j, k = n % dev.nx, (n // dev.nx) % dev.ny, n // (dev.nx * dev.ny)
        sub, glob, c = sub_device(dev, i, j, k)
        prob = solver.make_problem(sub)
        out[t] = 0.0 if dev.dir_id[n] >= 0 else prob.residual_full(phi[glob])[c]
    return out


def sampled_jv(dev, phi, v, nodes):
    """Oracle masked J(phi) v at the given nodes (identity rows on Dirichlet nodes)."""
    out = np.empty(len(nodes))
    vm = np.where(dev.dir_id >= 0, 0.0, v)
    for t, n in enumerate(nodes):
        n = int(n)
        if dev.dir_id[n] >= 0:
            out[t] = v[n]
            continue
        i, j, k = n % dev.nx, (n // dev.nx) % dev.ny, n // (dev.nx * dev.ny)
        sub, glob, c = sub_device(dev, i, j, k)
        prob = solver.make_problem(sub)
        out[t] = (prob.jacobian_full(phi[glob]) @ vm[glob])[c]
    return out


def ragged_device(stat="fd", T=4.0, volts=(1.5, 1.4, 0.5, 0.7, 0.3)):
    """A double-dot stack whose node counts leave ragged tiles in x, y and z."""
    dev = synth.double_dot_device("ragged", 37, 29, 19, np.asarray(volts, float),
                                  stat=stat, T_K=T)
    return dev


def full_charge_device(ionization="incomplete", volts=(2.1, 2.0, 1.1, 1.3, 0.9), stat="fd", T=4.0):
    """The ragged double-dot stack with the full space charge: holes, a
    1e15 cm^-3 boron substrate with the given ionization model, and the
    bottom contact at the oracle's Ohmic potential of that substrate."""
    from oracle import physics as ph
    dev = synth.with_species(ragged_device(stat=stat, T=T, volts=volts), ionization=ionization)
    st = ph.Statistics(stat, T, dev.m_eff, dev.Ec0_eV, holes=True, ionization=ionization)
    dev.dir_val[dev.contacts.index("bottom")] = ph.ohmic_potential(st, 0.0, synth.devices.NA_BULK_NM3)
    return dev
