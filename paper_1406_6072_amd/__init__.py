"""MI355X (gfx950) circulant-embedding generator of exact finite-survey
Gaussian fields, with lognormal + Poisson sampling and binned power spectra
(Carron, Wolk & Szapudi 2014, arXiv:1406.6072).

The compute path is the HIP library ``libcefield.so`` (C ABI in
``include/cefield.h``); ``binding`` marshals torch tensors and streams into it.
"""


def load():
    """Import the binding (raises ImportError if the library is not built)."""
    from . import binding
    return binding
