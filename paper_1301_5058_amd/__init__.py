"""MI355X-native explicit solver for the nutrient-chemotaxis bacterial colony
model of Leyva, Malaga and Plaza (arXiv:1301.5058).

The compute path is the HIP library ``libkc.so`` (C ABI declared in
``include/kc.h``); ``native`` binds it through ctypes and ``solver`` wraps it
for torch device tensors.  ``workload`` holds the seeded input recipes.
"""
__all__ = ["workload", "native", "solver"]
