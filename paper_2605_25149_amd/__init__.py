"""MI355X-native quasi-orthogonal inverse-operator eigensolver (HIP, gfx950).

The compute path lives in ``libqo_hip.so`` (hand-written HIP kernels behind a
C ABI declared in ``include/qo.h``); ``binding`` marshals arguments to it.
Importing the package loads nothing; ``binding`` loads the library on first use
and raises if it is missing.
"""

__all__ = ["binding", "inputs"]
