"""CPU float64 oracle for the multi-messenger Wiener filter.

TEST INFRASTRUCTURE ONLY.  Nothing on the GPU product path imports, calls or
links this package; it exists so tests, the smoke check and the CPU baseline of
the benchmark can compare the GPU library against a plain, slow and obviously
correct implementation written from the paper (Huffenberger 2017,
"Preconditioner-free Wiener filtering with a dense noise matrix").

Contents and what pins each part (tests marked ``not gpu``):

* ``bases``     pixel / 2-D Fourier / stripe-row bases.  Pinned by explicit DFT
                matrices and by dense covariance matrices built from explicit
                exponential sums (brute-force conditional minimisation).
* ``messenger`` setup, one sweep, residual, joint objective, schedules, solve
                (Section 2, Section 3.3 cooling, Appendix A).  Pinned by:
                each single update equals the exact minimiser of the dense joint
                quadratic (eqn 2mess_prob) in that field; the converged iterate
                equals the dense Cholesky Wiener solution; the stationary closed
                form; the one-step EW limit (Section 3.1); the joint objective
                never increases under a single update; rho -> 0 iff the
                chi^2 gradient vanishes; the profile identity min J = chi^2.
                It also holds the two-level merged chain and the augmented-signal
                chain (Appendix A shortcuts, ``Settings.chain``), pinned by
                reaching the dense solution's fixed point.
* ``direct``    the Wiener filter by its definition (dense Cholesky, closed
                form), chi^2 and its gradient.  Pinned by exact small cases
                (1-pixel algebra, white-noise-only Fourier closed form).
* ``warmnet``   the convolutional warm-start predictor (not from the paper:
                the iteration may start anywhere, Section 2): circular 3x3
                convolutions, pooling, upsampling, forward and reverse-mode
                gradient, Adam.  Pinned by brute-force loops, adjoint
                identities, translation equivariance and central finite
                differences of the loss.

Parity unpinned: the adaptive-schedule trajectory (lambda decisions depend on
rounding); tests replay a recorded lambda sequence as a fixed schedule instead.
"""

from . import bases, direct, messenger, warmnet  # noqa: F401
from .messenger import (  # noqa: F401
    AdaptiveSchedule,
    FixedSchedule,
    InvalidInput,
    NotPositiveDefinite,
    Settings,
    cooling_ramp,
    diagnostics,
    diagnostics_of_field,
    init_state,
    inverse_noise_weight,
    joint_objective,
    next_lambda,
    setup,
    solve,
    sweep,
)
