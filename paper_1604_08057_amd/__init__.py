"""MI355X-native two-sided Lanczos sign function of the Wilson-Dirac operator
at finite chemical potential and its gauge-link derivative (HIP, gfx950).

The computation lives in ``libtslov.so`` (C ABI in ``include/tslov.h``);
``paper_1604_08057_amd.tslov`` is the Python binding.
"""
from .tslov import Context, SignGrad, TslovError, TslovLibraryMissing, load_library  # noqa: F401
