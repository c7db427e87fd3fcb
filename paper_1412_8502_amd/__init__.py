"""MI355X (gfx950) implementation of the molecular-dynamics hot path of the
nuclear-pasta model of arXiv:1412.8502: pair forces (Eq. 1, Table I),
velocity Verlet in an expanding periodic box (Eq. 3) and the proton-linking
cluster algorithm (Sec. II.C), behind the C ABI of include/pasta.h.

``paper_1412_8502_amd.binding`` loads the HIP library (libpasta.so) and fails
loudly when it has not been built; ``paper_1412_8502_amd.inputs`` draws seeded
synthetic initial states.
"""
import importlib

__all__ = ["binding", "inputs", "autotune"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
