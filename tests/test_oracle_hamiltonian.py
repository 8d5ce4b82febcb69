"""Pins for the oracle's automaton Hamiltonian MPO (App. B.1).

The MPO, contracted to a dense matrix, must equal the Hamiltonian built
independently as a sum of Kronecker products (exact diagonalisation
module).  The bond dimensions are pinned to the values the paper prints.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as cf
from oracle import ed
from oracle import mpo as M

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _lattices():
    return [
        W.chain(6),
        W.random_couplings(W.chain(7), 1),
        W.with_couplings(W.chain(6), 1.0, 1.7),          # XXZ, Delta = 1.7
        W.with_couplings(W.chain(6), 1.0, 0.0),          # XY
        W.square_snake_obc(3, 3),
        W.square_cylinder(3, 3),
        W.triangular_yc(3, 3),
        W.random_couplings(W.square_cylinder(2, 4), 5),
    ]


@pytest.mark.parametrize("lat", _lattices(), ids=lambda l: l.name)
def test_mpo_equals_kronecker_sum(lat):
    H = M.hamiltonian(lat.n_sites, lat.bonds, lat.jxy, lat.jz)
    Hd = ed.xxz_dense(lat.n_sites, lat.bonds, lat.jxy, lat.jz)
    assert np.abs(M.to_dense(H) - Hd).max() < 1e-14


def test_golden_bond_dims():
    g = json.load(open(os.path.join(GOLD, "bond_dims.json")))
    lat = W.chain(12)
    assert max(M.automaton_bond_dims(lat.n_sites, lat.bonds)) == g["chain"]["D_H"]
    for Wd, dh in zip(g["square_obc_snake"]["W"], g["square_obc_snake"]["D_H"]):
        lat = W.square_snake_obc(Wd, 6)
        assert max(M.automaton_bond_dims(lat.n_sites, lat.bonds)) == dh
        assert max(j - i for i, j in lat.bonds) == 2 * Wd - 1


def test_traces_closed_form():
    lat = W.random_couplings(W.chain(7), 2)
    H = M.hamiltonian(lat.n_sites, lat.bonds, lat.jxy, lat.jz)
    assert abs(M.trace(H)) < 1e-12
    z0 = 2.0 ** lat.n_sites
    assert abs(M.trace_of_product(H, H) / z0 - cf.h2_per_state(lat.jxy, lat.jz)) < 1e-13
    assert abs(M.trace_of_product(H, H, H) / z0 - cf.h3_per_state(lat.jxy, lat.jz)) < 1e-13


def test_h3_closed_form_against_dense():
    lat = W.with_couplings(W.square_cylinder(3, 3), 0.8, 1.3)
    lat = W.Lattice(lat.name, lat.n_sites, tuple(b for b in lat.bonds if not (b[1] - b[0] == 2 and b[0] % 3 == 0)),
                    lat.jxy[:0], lat.jz[:0])
    # a triangle-free subset of bonds (drop the periodic wrap of each column)
    lat = W.Lattice(lat.name, lat.n_sites, lat.bonds, tuple([0.8] * len(lat.bonds)), tuple([1.3] * len(lat.bonds)))
    Hd = ed.xxz_dense(lat.n_sites, lat.bonds, lat.jxy, lat.jz)
    z0 = 2.0 ** lat.n_sites
    assert abs(np.trace(Hd @ Hd @ Hd) / z0 - cf.h3_per_state(lat.jxy, lat.jz)) < 1e-12
    assert abs(np.trace(Hd @ Hd) / z0 - cf.h2_per_state(lat.jxy, lat.jz)) < 1e-12


def test_xy_closed_form_vs_ed():
    """App. F's free-fermion partition function equals exact diagonalisation."""
    g = json.load(open(os.path.join(GOLD, "xy_chain.json")))
    J = g["J"]
    for L in (6, 9):
        lat = W.with_couplings(W.chain(L), J, 0.0)
        E = ed.spectrum(lat.n_sites, lat.bonds, lat.jxy, lat.jz)
        for beta in (0.1, 1.0, 7.0):
            assert abs(ed.lnZ(E, beta) - cf.xy_chain_lnZ(L, J, beta)) < 1e-11


def test_mpo_product_and_trace_helpers():
    lat = W.random_couplings(W.chain(5), 9)
    H = M.hamiltonian(lat.n_sites, lat.bonds, lat.jxy, lat.jz)
    Hd = M.to_dense(H)
    H2 = M.product(H, H)
    assert np.abs(M.to_dense(H2) - Hd @ Hd).max() < 1e-12
    Ht = M.transpose(H)
    assert np.abs(M.to_dense(Ht) - Hd.T).max() < 1e-14
    assert abs(M.inner(H, H) - np.sum(Hd * Hd)) < 1e-11
    assert abs(M.trace_of_product(H, H, H, H) - np.trace(Hd @ Hd @ Hd @ Hd)) < 1e-9
