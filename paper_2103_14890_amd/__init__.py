"""qcoll: MI355X-native fast spectral Boltzmann collision operator.

The product is libqcoll.so (C ABI declared in include/qcoll.h); the Python
binding in `qcoll` only marshals arguments. Import `paper_2103_14890_amd.qcoll`
to load the library (it raises if the library has not been built).
"""

__all__ = ["qcoll", "build"]
