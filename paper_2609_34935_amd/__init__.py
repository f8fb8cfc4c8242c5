"""MI355X trajectory simulator for amplitude-damped bucket-brigade QRAM
queries (qubit and qutrit encodings), pruned and full evolution, behind the C
ABI of include/qram.h."""
from .qram import (QRAM_MODE_FULL, QRAM_MODE_PLAIN, QRAM_MODE_PRUNED, QRAM_QUBIT, QRAM_QUTRIT,
                   STATS_DTYPE, QramContext, QramError, QramServer, load_library, qram_fidelity)

__all__ = ["QRAM_MODE_FULL", "QRAM_MODE_PLAIN", "QRAM_MODE_PRUNED", "QRAM_QUBIT", "QRAM_QUTRIT", "STATS_DTYPE",
           "QramContext", "QramError", "QramServer", "load_library", "qram_fidelity"]
