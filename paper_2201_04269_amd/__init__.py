"""Multi-baryon correlator contractions on MI355X (gfx950).

Determinant-form evaluation of two-point correlators of multi-baryon
operators (Humphrey, Detmold, Young, Zanotti, arXiv:2201.04269) behind the C
ABI of libmbc (include/mbc.h).  Submodules:

  api       IndexSet, Plan, contract, contract_backward, Contract (autograd)
  synth     seeded synthetic propagators
  build     in-tree hipcc build of libmbc.so
"""

__all__ = ["IndexSet", "Plan", "contract", "contract_backward", "Contract"]


def __getattr__(name):
    if name in __all__:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
