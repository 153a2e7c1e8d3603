"""MI355X-native G4 slice accumulation (one GPU's share of the DCA++ two-particle
Green's function update, arXiv 2105.00027).

The work is done by the HIP C-ABI library libg4.so (include/g4.h); the
binding lives in ``paper_2105_00027_amd.g4`` and is imported on first use so
that building the library does not require it to exist.
"""
import importlib

__all__ = ["g4"]


def __getattr__(name):
    if name == "g4":
        return importlib.import_module(__name__ + ".g4")
    raise AttributeError(name)
