"""Plain FP64 CPU oracle for the hierarchical-simulation CVA path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls or links
this package; only the tests, the smoke check and the benchmark's CPU-baseline leg
do.  It shares no code with the HIP library: the two sides meet only through the
seeded input arrays of the ``workloads`` module.

Each function follows the paper's definition of the quantity it computes, in the
paper's order, with NumPy FP64 arithmetic and no blocking or fusion beyond what
that definition states.  Where the paper is silent or garbled the docstring names
the reading taken.

Parity status of the functions (what pins each one, besides the GPU path):
  philox4x32_10          published known-answer vectors (tests/golden/philox_kat.txt)
  uniforms / normals     exact grid property, moments, KS against N(0,1)
  simulate_outer         Vasicek zero-coupon closed form, OU moments, FX martingale
  zc / swap_price        closed form at t=0 (par swap has zero value), martingale
  default dates          CIR survival closed form, literal rule on hand cases
  pathwise loss / T      exact conditional mean/variance, unbiasedness vs n_b=1,
                         brute-force enumeration on tiny inputs
  regression (BaseAlg)   least-squares refit == numpy lstsq; h=0 fit == lstsq;
                         one Adam step == hand-derived update
  sensitivities (FD)     convergence in h; analytic derivative of a closed form
  oversim (chooser)      R, Q recovered on a hierarchical sample of known variances; the
                         variance law's minimiser over a brute-force grid equals N*; the
                         proof's rearranged variance equals the direct one; l:ratio exact
  branch (nested / twin) prefix equals the outer path bitwise; CIR closed form of the
                         conditional survival increments; twin estimator unbiased on
                         samples of known conditional mean (e:val1 for B = 2); tower
                         property against independent outer paths
  alive-group targets    dead draws carry no loss; the alive group's sum of squares equals the
  (one counterparty)     weighted row's for any prediction; weight x target = inner average;
                         many draws approach the survival-conditioned conditional mean
  weighted regression    integer weights equal duplicated rows (loss, gradient, refit)
  per-sample rows        draw average = T; indicator increments = default counts; one
                         counterparty: per-sample loss = grouped alive loss + const; labels =
                         the loss definition as a double loop on a tiny case
"""
from . import philox, closed_forms, model, inner, pipeline, regression, sensitivities, oversim, branch  # noqa: F401
