"""Plain FP64 CPU oracle of the robust-SOCP inner solve (test infrastructure only).

This package is the checker, not the product: only the tests, the smoke entry
point and the benchmark's CPU-baseline leg may import it.  It shares no code
with the HIP library; both read problems from the `synth` generators.

Contents, each following the passage it cites (cuNRTO, arXiv 2603.02642):
  models     -- unicycle, quadrotor and joint-space arm dynamics with analytic
                Jacobians (supplementary "Dynamical Models"), 7-link DH kinematics
  linearize  -- nominal rollout, dense F_u / F_zeta, robust constraint data
                b_j, b_hat_j, g_j^0 (supplementary section I), QP data of Q_u
  soc        -- closed-form projection onto the second-order cone
                (supplementary section II-C, three cases in printed order)
  qp         -- the (delta_u, p) block: exact minimiser by semismooth Newton
                with exact line search and a bisected trust-region multiplier
  dr         -- NRTO-DR: ADMM over {k_v, p~} / {delta_u, p}, first block by
                relaxed Douglas-Rachford (Section III, supplementary II)
  fulladmm   -- NRTO-FullADMM (Section IV, Algorithm 1, supplementary III)
  kkt        -- one FP64 KKT residual of the tractable linearised problem
  scp        -- minimal successive-linearisation loop around the solves
  robust     -- closed-form worst case and Monte-Carlo disturbance checks
  mlp        -- FP64 reference MLP (GELU) with backward pass and Adam
  warm       -- DR state rebuilt from a predicted (du, p~, pi) and the cold
                fallback test (the learned warm start)

Parity pins live in tests/test_oracle_*.py.  Functions with no pin other than
the paper's own statement say "parity unpinned" in their docstring.
"""
