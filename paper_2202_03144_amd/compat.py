"""The paper's Python call pattern (Sec. 3.2, Fig. 3, Listing 1) over :class:`Plan`.

Step mode: ``<algo>init(...)`` creates the reconstruction, ``<algo>step()``
runs one iteration on the GPU, ``<algo>resobj()`` / ``<algo>resprobe()`` copy
the current object / probe back as NumPy arrays at any time, and
``<algo>post()`` releases everything.  Whole mode: ``<algo>(...)`` runs all
iterations and returns (object, probe).  Inputs are arrays rather than the
paper's command string: counts (J, N, N), positions (J, 2), object guess,
probe guess, plus iteration parameters as keywords.  ``<algo>init(cmd)``
with a command string instead (see :mod:`.command`) runs the paper's
simulation mode, as in Listing 1.
"""
from __future__ import annotations

from .plan import Plan, reconstruct

_current: dict = {}


def _init(algo, counts, positions=None, obj=None, probe=None, device=0, **params):
    _post(algo)
    if isinstance(counts, str):
        from .command import iteration_params, simulated_plan
        pl, g, _, _ = simulated_plan(counts, device=device)
        _current[algo] = (pl, {**iteration_params(g), **params})
        return
    pl = Plan(counts.shape[-1], probe.shape[0], counts.shape[0], obj.shape, device=device)
    pl.load_patterns(counts)
    pl.load_positions(positions)
    pl.set_object(obj)
    pl.set_probe(probe)
    _current[algo] = (pl, params)


def _plan(algo):
    if algo not in _current:
        raise RuntimeError(f"{algo}init() has not been called")
    return _current[algo]


def _step(algo, n=1):
    pl, params = _plan(algo)
    pl.iterate(algo, n, **params)


def _post(algo):
    if algo in _current:
        _current.pop(algo)[0].close()


def _whole(algo, counts, positions, obj, probe, n_iter, **params):
    o, p, _ = reconstruct(algo, counts, positions, obj, probe, n_iter, **params)
    return o, p


def epieinit(counts, positions=None, obj=None, probe=None, **params): _init("epie", counts, positions, obj, probe, **params)
def epiestep(n=1): _step("epie", n)
def epieresobj(): return _plan("epie")[0].object()
def epieresprobe(): return _plan("epie")[0].probe()
def epiepost(): _post("epie")
def epie(counts, positions, obj, probe, n_iter, **params): return _whole("epie", counts, positions, obj, probe, n_iter, **params)


def dminit(counts, positions=None, obj=None, probe=None, **params): _init("dm", counts, positions, obj, probe, **params)
def dmstep(n=1): _step("dm", n)
def dmresobj(): return _plan("dm")[0].object()
def dmresprobe(): return _plan("dm")[0].probe()
def dmpost(): _post("dm")
def dm(counts, positions, obj, probe, n_iter, **params): return _whole("dm", counts, positions, obj, probe, n_iter, **params)


def lsqmlinit(counts, positions=None, obj=None, probe=None, **params): _init("lsqml", counts, positions, obj, probe, **params)
def lsqmlstep(n=1): _step("lsqml", n)
def lsqmlresobj(): return _plan("lsqml")[0].object()
def lsqmlresprobe(): return _plan("lsqml")[0].probe()
def lsqmlpost(): _post("lsqml")
def lsqml(counts, positions, obj, probe, n_iter, **params): return _whole("lsqml", counts, positions, obj, probe, n_iter, **params)
