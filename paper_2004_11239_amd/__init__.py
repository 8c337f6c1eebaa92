"""MI355X-native fast Fourier spectral evaluation of the non-cutoff Boltzmann
collision operator (Hu & Qi, arXiv:2004.11239).

The compute path is the HIP library libbzq.so (C ABI in include/bzq.h); the
`bzq` module binds it for torch tensors.  Importing `bzq` fails if the
library has not been built (there is no CPU fallback).
"""
import importlib

__all__ = ["bzq", "build"]


def __getattr__(name):
    if name in ("bzq", "build", "serve"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
