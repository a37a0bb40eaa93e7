"""MI355X-native D3M factor/solve path (Moshfegh & Vouvakis, ICEAA 2016).

Thin Python layer over ``libd3m.so`` (the C ABI declared in
``include/d3m.h``): argument marshalling only.  Every step of the method
(assembly of the subdomain systems on the host; interior elimination,
assembly of K, block LDL^T with restricted Bunch-Kaufman pivoting and the
solve sweeps on the GPU) runs inside the library.  PyTorch supplies device
memory and streams.  There is no fallback: if the library is missing, import
fails.
"""
from ._lib import (D3MError, Solver, FP64, FP32_IR, KERNEL_IDS, library_path,
                   exported_symbols)
from .autograd import D3MSolve
from .autotune import autotune

__all__ = ["D3MError", "Solver", "FP64", "FP32_IR", "KERNEL_IDS", "D3MSolve", "autotune",
           "library_path", "exported_symbols"]
