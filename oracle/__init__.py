"""FP64 CPU oracle for the #DNN-Verification counter with Symbolic Linear Relaxation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or execute this
package: only the tests, the smoke check and the benchmark's CPU-baseline leg use it.  It
shares no code with the HIP engine (no kernels, headers, helpers or constants); both read
their inputs from the separate ``synth`` generator.

Everything here is plain, slow and written to be checked against the paper by eye:

* ``slr``     symbolic propagation of a lower and an upper linear equation per neuron through
              a ReLU network (paper §2.2 and §3), the relaxation of Eq. 1 at crossing ReLUs,
              concretization over a box, the property test of §3, plus a pure-Python
              per-box twin and a concrete forward pass.
* ``count``   Alg. 1 (exact count) as a level-synchronous breadth-first branch-and-bound with
              exact dyadic volume accounting, and the CountingProVe-style approximate count
              used with it as the leaf backend (§2.3, §4).
* ``philox``  the Philox4x32-10 counter-based generator (Salmon et al., SC 2011), which both
              sides implement from its published definition for the random draws of the
              approximate count.

Where the paper is silent or garbled the readings are:
  one ratio u/(u-l) for both equations of Eq. 1, with l the concrete minimum of the lower
  equation and u the concrete maximum of the upper one; a dead ReLU (u <= 0) zeroes both
  equations, an active one (l >= 0) keeps them; the property C y + d > 0 (all rows) is the
  unsafe set and is folded into the last affine layer; a box is unsafe when every row's lower
  bound is > 0, safe when some row's upper bound is <= 0, otherwise it is bisected at the
  midpoint of its widest side (lowest index on ties); the count adds the input-box volume
  |X| (not the output set) of unsafe leaves; the search stops at a maximum depth or, at a
  level boundary, at a leaf budget, and reports the bracket [unsafe, unsafe + undecided].

Every bound carries an FP64 rounding margin (Higham's gamma_n = n u / (1 - n u), u = 2^-53),
so the computed bounds are sound for the exact network; the margin is ~1e-13 relative.
"""
from . import slr, count, philox, alpha  # noqa: F401
