"""Plain FP64 CPU oracle for block belief propagation (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls, links or imports it, and
it shares no code with the library: the two implement the same readings of the
paper independently.

Modules
-------
``blockbp``  block-BP message updates, residual, observables, log-norm.
``brute``    brute-force state vector and exact strip contraction (pins).
``plain_bp`` plain BP with single-site blocks (pin for the orientation logic).
"""
