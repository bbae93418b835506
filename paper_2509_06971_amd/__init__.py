"""MI355X (gfx950) implementation of the pseudo-transient topology-optimisation
hot path: accelerated pseudo-transient relaxation of linear elasticity and heat
conduction on a staggered grid, the compliance sensitivity and the phase-field
design update, behind the C ABI of include/petto.h."""
from . import _lib  # noqa: F401

__all__ = ["Context", "ComplianceFn", "load_library"]


def load_library():
    return _lib.load()


def __getattr__(name):
    if name in ("Context", "ComplianceFn"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
