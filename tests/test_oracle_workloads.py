"""Checks of the seeded workloads against the oracle: sizes match the unique
and element-local DOF counts, the time step is stable for the SIPG operator,
and the PMUT coupling strength stays in the range where the synchronised
explicit coupling is stable."""
import numpy as np
import pytest

from oracle import ref
from paper_2603_06267_amd import workloads as W


def test_dof_counts():
    assert W.unique_dofs(W.config1()) == 4913 and W.element_local_dofs(W.config1()) == 8000
    assert W.unique_dofs(W.config2()) == 132450 and W.element_local_dofs(W.config2()) == 259072
    assert W.unique_dofs(W.config3()) == 32822146 and W.element_local_dofs(W.config3()) == 73007104


@pytest.mark.parametrize("cfg", [1, 2])
def test_stability_and_coupling(cfg):
    wl = W.CONFIGS[cfg]()
    s = ref.from_workload(wl, shape_fn=W.shape_fn(wl))
    lam = s.lambda_max(150)
    assert s.dt ** 2 * lam / 4 < 0.8
    M = s.mass()
    kappa = wl["domains"][0]["rho"] * wl["domains"][0]["c"] ** 2
    X = []
    for k in range(min(s.Np, 4)):
        for m in range(s.Nm):
            nd, v = s.coupling(k, m)
            X.append(kappa * s.dt ** 2 * np.sum(v ** 2 / M[nd]))
    assert 0.01 < max(X) < 1.0
