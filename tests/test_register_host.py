"""Host-side step of the registration loop (no GPU): pot_rigid_align, the
rotation of the weighted Procrustes problem by Horn's quaternion method,
against the oracle's SVD form of the appendix (oracle/register.py)."""
import os

import numpy as np
import pytest


def _lib_or_skip():
    from paper_2601_17196_amd import pot
    if not os.path.exists(pot.lib_path()):
        pytest.skip("libpot.so not built")
    return pot


@pytest.mark.parametrize("seed", range(8))
def test_rigid_align_matches_the_svd_form(seed):
    pot = _lib_or_skip()
    from oracle import register as G
    g = np.random.default_rng(seed)
    X = g.normal(size=(25, 3))
    Y = g.normal(size=(17, 3)) if seed % 2 else X[:17] * np.array([1.0, 1.0, -1.0])   # mirror-like cases too
    P = g.uniform(size=(25, 17))
    _, _, H, _ = G.plan_moments(X, Y, P)
    Ro, _ = G.procrustes(X, Y, P)
    R = pot.rigid_align(H)
    assert np.max(np.abs(R - Ro)) <= 1e-12
    assert abs(np.linalg.det(R) - 1.0) <= 1e-12 and np.max(np.abs(R @ R.T - np.eye(3))) <= 1e-12


def test_rigid_align_exact_rotation():
    pot = _lib_or_skip()
    from tests.test_oracle_pins import _rot
    for k, ang in enumerate((0.0, 0.3, 1.5, 3.1)):
        R0 = _rot([1.0, -2.0, 0.5 + k], ang)
        Y = np.random.default_rng(k).normal(size=(30, 3))
        H = (Y @ R0.T).T @ Y          # sum_j x_j y_j^T with x_j = R0 y_j
        assert np.max(np.abs(pot.rigid_align(H) - R0)) <= 1e-12
