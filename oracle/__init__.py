"""FP64 CPU oracle for the transmission forward model and its chi^2 gradient.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct reference that the HIP library is checked against.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it;
the library itself never routes through it.  It shares no code with the HIP
path: it reads the same seeded input arrays (``synth``) and nothing else.

Every function follows a passage of Al-Refaie et al., "TauREx 3: A fast,
dynamic and extendable framework for retrievals" (arXiv:1912.07759), cited by
section and equation.  Where the paper is silent or ambiguous the reading
used is stated in the function's docstring.

Pinning status (what fixes each function other than itself) is listed in
``oracle/forward.py``'s module docstring.
"""

from .forward import (  # noqa: F401
    pressure_grid, chemistry, altitude, shell_boundaries, chord_lengths,
    annulus_weights, bracket, interp_xsec, interp_cia, number_density,
    opacity, optical_depth, transit_depth, native_bin_edges, bin_weights,
    bin_spectrum, forward_model, forward_batch, chi2, two_layer_vmr, chemistry_profile,
    model_chemistry,
)
from .adjoint import chi2_and_grad, chi2_grad_batch  # noqa: F401
from .emission import (emission_model, emergent_intensity, gauss_legendre_mu,  # noqa: F401
                       planck, vertical_optical_depth)
