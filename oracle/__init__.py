"""CPU oracle for the DDM image structure function (arXiv 2012.05695).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
anything in this package; only the test suite, the smoke check and the CPU
baseline leg of the benchmark do.  The GPU library shares no code, table or
helper with it.

What it computes, in FP64, deliberately slowly and by definition:

* ``dft``       -- the unnormalised forward 2-D DFT of each frame on the
                   non-redundant half plane, written out as a naive separable
                   sum (no FFT).  Section "The algorithm", the 2-D transform
                   that Eq. (1) applies to image differences.
* ``structure`` -- the image structure function of Eq. (1) by direct
                   differences of the transformed frames (indices read as
                   I_n - I_{n-m}; see the module docstring there).
* ``radial``    -- azimuthal averaging of D over integer |q|^2 bins.
* ``lm``        -- Levenberg-Marquardt fit of D = A(1-exp(-m/tau)) + B.
* ``mlp``       -- forward/backward of the fit-initialisation network.

Pins that tie these functions to the paper and to mathematics live in
``tests/test_oracle_*.py``.
"""

from .dft import dft_half_plane, dft_columns, q_list, k2_of
from .structure import structure_function_direct, structure_function_sum_rule_rhs
from .radial import radial_average, bin_index

__all__ = [
    "dft_half_plane",
    "dft_columns",
    "q_list",
    "k2_of",
    "structure_function_direct",
    "structure_function_sum_rule_rhs",
    "radial_average",
    "bin_index",
]
