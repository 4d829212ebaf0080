"""MI355X-native NEP energy / force / virial engine (hand-written HIP for gfx950).

Layers:
  csrc/      HIP kernels and the C-ABI (include/nep.h) -> libnep.so
  binding    ctypes marshalling of the C-ABI, same names as the header
  engine     device-resident systems (torch owns the memory, libnep computes):
             Replica (evaluation, MD with ensembles, strain, HNEMD and the
             constrained label runs), FitnessBatch (many structures x many
             parameter sets in one persistent launch), SnesTrainer (the SNES
             training loop on the device), MdStepBatch and Server (continuous
             batching of resident MD replicas)
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnep.so")

__all__ = ["LIB_PATH"]
