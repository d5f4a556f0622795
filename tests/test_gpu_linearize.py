"""GPU parity of the device constraint-data formation (nrto_linearize: rollout,
analytic Jacobians, adjoint recursion) against the oracle's dense definition
(impulse-built F_u, F_zeta; b_j = F_u' grad g_j, b_hat_j = r F_zeta' grad g_j)."""
import numpy as np
import pytest

import synth
from oracle import linearize

from helpers import compact_socp, rel_err

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _perturbed(prob, seed, scale):
    d = synth.Draws(seed)
    prob.u_init = prob.u_init + scale * d.u(prob.u_init.size, -1, 1).reshape(prob.u_init.shape)
    return prob


# The quadrotor's torques act on J = 0.01 I: a torque perturbation of 0.3 spins it up to
# ~9 rad/s and its rollout then amplifies a 1e-15 relative change of the controls to
# 5e-7 in the states (1e-14 at 0.01), so its nominal controls are perturbed by 0.01.
@pytest.mark.parametrize("make,T,scale", [(synth.config1, 20, 0.5), (synth.config2, 50, 0.01),
                                          (synth.config3, 12, 0.5)])
def test_linearize_matches_oracle(make, T, scale):
    _torch()
    from paper_2603_02642_amd import nrto
    prob = make()
    prob.T = T
    prob.u_init = prob.u_init[:T]
    prob = _perturbed(prob, 5, scale)
    s = linearize.assemble(prob, prob.u_init, 2.0)
    ref = compact_socp(s)
    c = nrto.Context([prob])
    c.linearize()
    got = c.download_socp(0)
    for k in ["A", "B", "xhat", "uhat", "g0", "w", "bhat", "bvec"]:
        e = rel_err(got[k], np.asarray(ref[k]).ravel())
        assert e <= 1e-12, (k, e)
