"""Plain, slow, FP64 CPU oracle of the learnable-differentiable finite-volume
step (Yan et al., "Learnable-Differentiable Finite Volume Solver for
Accelerated Simulation of Flows", KDD 2025).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, header,
table or constant generator with the HIP library; the only module both sides
use is ``synthetic_inputs`` (seeded random fields and weights, no method
arithmetic).

Every function follows the paper's definitions step by step in float64
(torch CPU ops, so that autograd gives reference vector-Jacobian products):

* ``fv``          finite-volume residuals (Sec. 3.3 Eqs. 3-4, App. B.2 S1-S7)
* ``projection``  MAC divergence, gradient, spectral Poisson solve, projection
                  (App. B.3 S8-S10, App. B.4 S11-S14)
* ``timestep``    RK4 with a projection per sub-step (Sec. 3.2, App. B.5
                  S15-S20) and SSP-RK3 for the Burgers configuration
* ``cnn``         the 3x3 convolutional coefficient network (the learnable
                  flux block in per-cell form, Sec. 3.4 Eqs. 5-7)
* ``learned``     sum-to-one coefficient constraint, temporal correction and
                  the learned step (Eq. 2, Sec. 3.5)
* ``fno``         the Fourier neural operator of the flux block's frequency
                  part (Sec. 3.4 Eq. 8; Li et al. 2021)
* ``fluxblock``   the paper's flux block O_P + O_L + O_F (uniform learnable
                  5x4 kernels and FNO fields, Sec. 3.4 Eqs. 5-8) in the step,
                  and the temporal correction block (Eq. 2)
* ``scalar``      the passive scalar of the shear-flow system, stepped with
                  the velocity's RK4 stages
* ``ic``          seeded initial conditions (App. C.1, S30-S31)
* ``rng``         SplitMix64 and Box-Muller, from their published definitions
* ``metrics``     down-sampling, vorticity, RMSE/MAE/MNAD/HCT/PCC (App. D.1,
                  S32-S36)
* ``optim``       MSE rollout loss (Eq. 13) and Adam

Parity status: every function is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` against closed forms, invariants, brute force or
library special cases, except where a module header says "parity unpinned".
"""
