"""MI355X-native thermal two-component Shan-Chen lattice Boltzmann update
(TLBfind, arXiv:2109.12565) behind the C ABI of ``include/tlb.h``.

``Simulation`` wraps one handle of the HIP library ``lib/libtlb.so``.
"""
from ._lib import EXPORTS, PRECISIONS, Simulation, TlbError, load_library, top_nusselt_loss

__all__ = ["EXPORTS", "PRECISIONS", "Simulation", "TlbError", "load_library", "top_nusselt_loss"]
