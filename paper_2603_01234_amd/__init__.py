"""MI355X-native NEP energy / force / virial engine (hand-written HIP for gfx950).

Layers:
  csrc/      HIP kernels and the C-ABI (include/nep.h) -> libnep.so
  binding    ctypes marshalling of the C-ABI, same names as the header
  engine     device-resident systems (torch owns the memory, libnep computes)
  batch      many structures x many parameter sets in one persistent launch
  serve      continuous-batching MD server over resident replicas
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnep.so")

__all__ = ["LIB_PATH"]
