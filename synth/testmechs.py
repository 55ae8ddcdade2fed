"""Small mechanisms with closed-form solutions (inputs of the integrator pins).

* ``isomerisation``: A <=> B, unimolecular, equal heat capacities, formation
  enthalpies and molar masses, so T and the density stay constant and
  Y_A(t) = Y_A,eq + (Y_A0 - Y_A,eq) exp(-(k_f + k_r) t) with
  K_c = exp(S_B/R - S_A/R).
* ``bimolecular``: P2 + Q2 (+ M) <=> 2 PQ with equal molar masses and
  enthalpies (constant T, moles and density) and a huge entropy gain so the
  reverse rate is negligible: second-order kinetics
  [A](t) = [A]0 D / ([B]0 exp(D k t) - [A]0), D = [B]0 - [A]0, with k the
  rate constant times [M] when a third body is present.  An inert species X
  with efficiency 3 keeps [M] constant but different from the total
  concentration.
"""
from __future__ import annotations

import numpy as np

from .mechfile import Mechanism


def _flat_nasa(cp_r, a7):
    return [cp_r, 0.0, 0.0, 0.0, 0.0, 0.0, a7]


def isomerisation(kf=2.0e5, dS_R=np.log(3.0), Ta=0.0, b=0.0):
    nasa = np.array([_flat_nasa(3.5, 10.0), _flat_nasa(3.5, 10.0 + dS_R)])
    return Mechanism(
        name="iso_A_B", seed=0, elements=["X"], element_mass=np.array([10.0]), species=["A", "B"],
        molar_mass=np.array([10.0, 10.0]), composition=np.array([[1], [1]]), nasa7=nasa,
        reaction_type=np.array([0]), nu_reac=np.array([[1, 0]]), nu_prod=np.array([[0, 1]]),
        arrhenius=np.array([[kf, b, Ta]]), efficiency=np.ones((1, 2)), falloff_low=np.zeros((1, 3)),
        troe=np.zeros((1, 4)))


def bimolecular(k=3.0e12, third_body=False, eff_inert=3.0):
    # species P2, Q2, PQ, X(inert); elements P, Q, Z all of mass 10 -> W = 20 for all
    nasa = np.array([_flat_nasa(3.5, 0.0), _flat_nasa(3.5, 0.0), _flat_nasa(3.5, 30.0), _flat_nasa(3.5, 5.0)])
    eff = np.ones((1, 4))
    eff[0, 3] = eff_inert
    return Mechanism(
        name="bimol_P2_Q2" + ("_M" if third_body else ""), seed=0, elements=["P", "Q", "Z"],
        element_mass=np.array([10.0, 10.0, 10.0]), species=["P2", "Q2", "PQ", "X"],
        molar_mass=np.array([20.0, 20.0, 20.0, 20.0]),
        composition=np.array([[2, 0, 0], [0, 2, 0], [1, 1, 0], [0, 0, 2]]), nasa7=nasa,
        reaction_type=np.array([1 if third_body else 0]), nu_reac=np.array([[1, 1, 0, 0]]),
        nu_prod=np.array([[0, 0, 2, 0]]), arrhenius=np.array([[k, 0.0, 0.0]]), efficiency=eff,
        falloff_low=np.zeros((1, 3)), troe=np.zeros((1, 4)))
