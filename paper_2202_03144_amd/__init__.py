"""ptymi: multi-mode ptychographic reconstruction (ePIE, DM, LSQML) on MI355X.

The reconstruction runs in hand-written HIP kernels for gfx950 behind the C
ABI of ``include/ptymi.h`` (``libptymi.so``, built in-tree by
:mod:`paper_2202_03144_amd.build`).  :class:`Plan` is the step-mode front end
(Sec. 3.2 of the ptychopy paper: initialise, iterate, fetch object and probe
at any time, release); :func:`reconstruct` is the whole mode; the
``epieinit / epiestep / ...`` functions mirror the paper's Python API.
"""
from ._lib import DM, EPIE, LSQML, PtyError  # noqa: F401
from .plan import Batch, Plan, reconstruct  # noqa: F401
from .compat import (  # noqa: F401
    dminit, dmpost, dmresobj, dmresprobe, dmstep,
    epieinit, epiepost, epieresobj, epieresprobe, epiestep,
    lsqmlinit, lsqmlpost, lsqmlresobj, lsqmlresprobe, lsqmlstep,
    epie, dm, lsqml,
)

__all__ = ["Plan", "Batch", "reconstruct", "PtyError", "EPIE", "DM", "LSQML"]
