"""FP64 CPU oracle for ptychographic reconstruction (test infrastructure only).

This package is the plain, slow, obviously correct reference against which the
HIP path is checked.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark import it; the product library never does, and the two
share no code (only the seeded input generator in ``ptysynth`` serves both).

Every function works in complex128 / float64 with NumPy and ``scipy.fft`` and
follows the paper's methods (Sec. 2.3: ePIE, DM and LSQML reconstruct object
and probe from far-field diffraction patterns of overlapping scan positions,
with multi-mode probes, a probe-update start iteration and optional initial
guesses; Sec. 3.2: patterns are normalised at initialisation) and the cited
papers for the update rules.  See :mod:`oracle.ptycho` for the notation.

Parity status of each function is stated in its docstring; all are pinned by
the ``-m "not gpu"`` tests except where the docstring says "parity unpinned".
"""
from .ptycho import *  # noqa: F401,F403
from .ptycho import __all__  # noqa: F401
