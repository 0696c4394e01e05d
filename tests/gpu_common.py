"""Shared helpers of the GPU parity tests: seeded inputs (from the generator)
go to both the oracle and the HIP library; expected values come from the
oracle only."""
import numpy as np

from oracle import ks_oracle as ko
from paper_2106_03872_amd import synth


def oracle_ham(sysm, ecut=None):
    spec = sysm.spec
    g = ko.Grid(spec.n, spec.L, spec.ecut if ecut is None else ecut)
    atoms = [sysm.proj.atom(i) for i in range(spec.natoms)]
    return ko.Hamiltonian(g, sysm.vloc, atoms, sysm.proj.d)


def orbitals_device(spec, norb=None):
    """Generator coefficients scattered into a device box [norb, n0, n1, n2]."""
    import torch
    sel, vals = synth.orbital_values(spec, norb)
    out = torch.zeros((vals.shape[0], spec.npoints), dtype=torch.complex128, device="cuda")
    out[:, torch.from_numpy(sel).to("cuda")] = torch.from_numpy(vals).to("cuda")
    return out.reshape((vals.shape[0],) + tuple(spec.n))


def rel_err(a, b):
    """max over orbitals of ||a - b|| / ||b||"""
    a = np.asarray(a).reshape(a.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))
