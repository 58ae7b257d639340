"""FP64 brute-force CPU reference for the probe-plane rasterizer.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package: only the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP path; both sides are
fed by the seeded input generators in ``paper_2505_05643_amd.synth``, which
hold none of the method's arithmetic.

Every function evaluates the paper's definitions directly (UltraGauss,
Section 4.1 Eq. 5-9, Section 4.2 Eq. 11, Section 4.3 Eq. 12-13): every
Gaussian is evaluated at every 3D pixel point of every plane, in float64,
with no boxes, tiles or culling.

Pinning (see ``tests/test_oracle*.py``): closed forms, a library density,
invariants, brute-force ellipsoid sampling and finite differences fix every
function here.  The one part that is not pinned to a unique value is which
of several correct outputs a pixel takes when a pair sits on the cut-off
d^2 = chi^2 to within rounding: ``ambiguity`` reports the interval instead.
"""
from . import box_support, densify, params, quality
from .render import (CHI2_PAPER, Params, activate_l, covariance, sigmoid,
                     plane_points, render, render_points, grad, grad_points,
                     ambiguity_points, box_eq13, inplane_conic, d2_points,
                     sample_gaussian)

__all__ = ["box_support", "densify", "params", "quality", "CHI2_PAPER", "Params", "activate_l", "covariance", "sigmoid",
           "plane_points", "render", "render_points", "grad", "grad_points",
           "ambiguity_points", "box_eq13", "inplane_conic", "d2_points",
           "sample_gaussian"]
