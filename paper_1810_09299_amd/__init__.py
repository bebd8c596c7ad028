"""MI355X-native axisymmetric Allen-Cahn MRT lattice Boltzmann hot path
(Liang, Li, Chen & Xu, arXiv:1810.09299).

Submodules load lazily so that the seeded input generators (inputs) import
without the HIP library or a GPU:
  inputs  seeded case parameters and initial phase fields
  abi     ctypes binding of liblbm_axi.so (include/lbm_axi.h)
  case    AxiCase: one device-resident case (torch for memory and streams)
  batch   Batch: many cases advanced by one launch per step
  build   hipcc build of liblbm_axi.so
"""
import importlib

__all__ = ["inputs", "abi", "case", "batch", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
