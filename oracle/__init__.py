"""CPU FP64 oracle for SFFT image subtraction -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this package.  The product path (the HIP library and its Python
binding) never imports, links or calls it, and this package imports nothing
from the product path.
"""
from .sfft_oracle import *  # noqa: F401,F403
from . import mlp_oracle  # noqa: F401,E402
from .kernel_oracle import (apply_kernel, centre_kernel, convolve, decorrelation_kernel,  # noqa: F401,E402
                            decorrelation_spectrum, DECORR_GRID)
from . import ratio_oracle  # noqa: F401,E402
from .ratio_oracle import kernel_sums, ratio_constraints, ratio_map, solve_const_ratio  # noqa: F401,E402
from . import align_oracle  # noqa: F401,E402
from . import outmask_oracle  # noqa: F401,E402
from .outmask_oracle import fit_outmask, masked_rows, normal_system_outmask  # noqa: F401,E402
