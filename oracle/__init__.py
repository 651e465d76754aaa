"""FP64 CPU oracle for the CP-structured Bellman backup -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The GPU library never calls it, and it shares no
code with the GPU library: the only common module is the seeded instance
generator (``paper_2103_00331_amd.instances``), which builds inputs and holds
none of the solver's arithmetic.

Representations of the operator P_a, all in FP64:
  * ``dense``      (O1) -- P_a expanded to an explicit S x S matrix as the sum
                    of Kronecker products of the factors; value iteration,
                    policy iteration with an exact linear solve, brute-force
                    policy enumeration.  Tiny state spaces only.
  * ``sparse``     (O2) -- the per-state successor lists of Def. 3 (every
                    (s, s', P(s'|s,a)) with P > 0), stored as CSR; iterative
                    value iteration and policy iteration.  Shift/identity
                    factors (GridWorld) up to millions of states.
  * ``structured`` (O3) -- mode products of the value tensor with each factor
                    (numpy tensordot), one rank term at a time; any factors.
  * ``tt``         (O4) -- Tensor-Train and Tucker transition models (Sec. 5)
                    expanded to dense P_a from their definitions, for O1.
  * ``cpfit``      (O5) -- CP-ALS (Kolda & Bader 2009) fitting rank-R CP
                    factors to a tabular P_a (the decomposition step of Sec. 3).

Readings of the paper that the oracle fixes (the paper is silent on them):
  * state order of Def. 2 = row-major, last dimension fastest;
  * T[i, j] = P(next coordinate j | current coordinate i), contracted over j;
  * terminal states: V(s) = R(s), continuation masked;
  * greedy policy: lowest action index whose Q is within
    tol = 1e-12 * max(1, ||V||_inf) of the maximum (``common.greedy``);
  * policy improvement keeps the incumbent action unless another action beats
    it by more than tol; policy iteration stops when the policy is unchanged
    (Sec. 2.1).
"""
from . import common, cpfit, dense, mlp, sparse, structured, tt  # noqa: F401
from .common import greedy, improve, tie_tolerance  # noqa: F401
